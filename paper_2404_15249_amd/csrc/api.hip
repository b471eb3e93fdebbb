// C ABI of the KFBI library (see include/kfbi.h): contexts, problems, the
// operator apply, the device-resident GMRES solve and the step entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <queue>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "kfbi.h"
#include "batch.h"
#include "gmres.h"
#include "graph.h"
#include "kernels.h"
#include "plan.h"
#include "api_common.h"

using namespace kfbi;

GraphRec*& kfbi::graph_rec() {
    static thread_local GraphRec* rec = nullptr;
    return rec;
}

LaunchEvents& kfbi::launch_events() {
    thread_local LaunchEvents ev;
    return ev;
}

std::string& kfbi::last_error() {
    static thread_local std::string err;
    return err;
}

// ---------------------------------------------------------------- scratch of kfbi_apply_noalloc
//
// The entry point for callers that cannot allocate takes its scratch (the
// spline second derivatives, corrections and partial sums of one K_D apply)
// from this file-scope array instead of the problem's workspace.  Each device
// holds its own copy for the life of the process; host code uses the address
// hipGetSymbolAddress gives for it on that device (resolved once per device,
// when a context is created there), never the array's name.
constexpr size_t kNoAllocBytes = size_t(32) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};

// The scratch's address on `device` (the current device), resolved on first use.
kfbi_status scratch_on(int device, void** out) {
    if (device < 0 || device >= kMaxDevices) return kfbi::set_err(KFBI_ERR_UNSUPPORTED, "device index too large");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[device]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            hipGetLastError();
            return kfbi::set_err(KFBI_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        }
        g_scratch[device] = ptr;
    }
    *out = g_scratch[device];
    return KFBI_OK;
}
}  // namespace

struct kfbi_prob {
    kfbi_ctx* ctx = nullptr;
    Plan plan;
    double kappa = 0, tol = 1e-10;
    int restart = 50, max_iter = 500;
    double reorth = kGmReorthDefault;   // second Gram-Schmidt pass when |z| < reorth |w|
    int N = 0, n = 0, M = 0, Q = 0, I = 0;
    int Rm = 8, G = 1;           // sine modes per sparse-fast-solve workgroup; workgroups = ceil(n / Rm)
    DevPlan dp{};                // the double-layer operator's view (see plan_view)
    const double* cp_wn = nullptr;   // 6 M: weights of d_n v+ at the samples (the Neumann operator)
    std::vector<void*> allocs;
    size_t bytes = 0;
    // work buffers
    double* corr = nullptr;      // I
    double* corr_il = nullptr;   // T x 64: corrections in the interleaved layout of the sparse sums
    double* partial = nullptr;   // G M
    double* R = nullptr;         // N N
    double* A = nullptr;         // N N
    int precision = KFBI_FP64, refine = 0;
    float* X32 = nullptr;        // N N: FP32 transform storage (KFBI_FP32_REFINED)
    double* D = nullptr;         // N N: a refinement correction (refine_steps >= 2)
    int dstB = 8;                // columns per workgroup of the column transforms
    int Gcap = 1;                // workgroups the partial buffer has room for
    double* tmpM = nullptr;      // M
    double* partial_b = nullptr; // M x Gs: partials of the batched fast solve (allocated on first admission)
    int Gs = 0;
    const double* b_fgrid = nullptr;   // right-hand side of the batched request (caller owned)
    const double* b_fgam = nullptr;
    double* s2a = nullptr;       // M: spline second derivatives (density)
    double* s2b = nullptr;       // M: spline second derivatives (f on Gamma)
    int* d_flag = nullptr;       // 1: the density checked by a kfbi_apply call holds a NaN or Inf
    int h_flag = 0;              // its host copy
    GmresBufs gm{};
    GmresState st_host{};        // host copy of the GMRES state (stable address for async copies)
    GmresState* st_pub = nullptr;   // pinned host mirror the device publishes the state to (gm.pub)
    // timing: a start and an end event for each of an apply's three launches,
    // read back by kfbi_apply_timing
    static constexpr int kMaxTimed = 4096;
    bool timing = false;
    std::vector<hipEvent_t> ev;
    int t_count = 0;
    double tuned_apply_us = 0, tuned_grid_us = 0;
    // a captured batch of GMRES steps (apply + Arnoldi update) per operator
    // (kOpD, kOpN), replayed per batch
    // graphs of 32, 16, 8, 4, 2 and 1 steps (index k: kGraphSteps >> k
    // steps), so a run launches exactly the steps it has left, in few graphs
    static constexpr int kGraphSteps = 32;
    static constexpr int kGraphSizes = 6;
    hipGraphExec_t gexec[2][kGraphSizes] = {};
    bool graph_failed[2][kGraphSizes] = {};
    // Richardson and BiCGSTAB (Table 2's alternatives): vectors, state, and a
    // graph of a batch of iterations for each
    IterBufs ib{};
    hipGraphExec_t iexec[2] = {nullptr, nullptr};
    bool iexec_failed[2] = {false, false};
};

namespace {

template <class T>
kfbi_status dev_alloc(kfbi_prob* p, T** out, size_t count) {
    void* ptr = nullptr;
    const size_t b = std::max<size_t>(count, 1) * sizeof(T);
    if (hipMalloc(&ptr, b) != hipSuccess) {
        hipGetLastError();
        return set_err(KFBI_ERR_OOM, "device allocation of " + std::to_string(b) + " bytes failed");
    }
    p->allocs.push_back(ptr);
    p->bytes += b;
    *out = static_cast<T*>(ptr);
    return KFBI_OK;
}

template <class T>
kfbi_status upload(kfbi_prob* p, const T** out, const std::vector<T>& v) {
    T* d = nullptr;
    kfbi_status s = dev_alloc(p, &d, v.size());
    if (s) return s;
    if (!v.empty()) HIP_TRY(hipMemcpy(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    *out = d;
    return KFBI_OK;
}

void free_prob(kfbi_prob* p) {
    for (void* a : p->allocs) hipFree(a);
    p->allocs.clear();
    if (p->st_pub) hipHostFree(p->st_pub);
    p->st_pub = nullptr;
    p->gm.pub = nullptr;
    for (auto& e : p->ev)
        if (e) hipEventDestroy(e);
    p->ev.clear();
    for (auto& row : p->gexec)
        for (auto& g : row) {
            if (g) hipGraphExecDestroy(g);
            g = nullptr;
        }
    for (auto& g : p->iexec) {
        if (g) hipGraphExecDestroy(g);
        g = nullptr;
    }
}

// Per-mode constants of the x-direction tridiagonal systems (Alg. 4), FP64.
std::vector<ModeConst> mode_constants(int N, double h, double kappa) {
    std::vector<ModeConst> mc(N);
    for (int l = 1; l < N; ++l) {
        const double s = std::sin(M_PI * l / (2.0 * N));
        mc[l] = row_solve_constants(h * h * kappa + 4.0 * s * s, N);
    }
    return mc;
}

// The two boundary operators: K_D (the density is [v], the samples get v+) and
// K_N (the density is [d_n v], the samples get d_n v+).
enum Op { kOpD = 0, kOpN = 1 };

// The plan as one kernel sequence sees it: which jump the density is, and
// whether the interpolation extracts v+ or d_n v+ (the six weights it uses).
DevPlan plan_view(const kfbi_prob* p, bool normal_jump, bool normal_deriv) {
    DevPlan d = p->dp;
    d.normal_jump = normal_jump ? 1 : 0;
    if (normal_deriv) d.cp_w = p->cp_wn;
    return d;
}

DevPlan op_view(const kfbi_prob* p, int op) { return plan_view(p, op == kOpN, op == kOpN); }

// bytes of one complex pair in the column transforms of a precision mode
size_t cpx_bytes(int precision) { return precision == KFBI_FP64 ? 2 * sizeof(double) : 2 * sizeof(float); }


// Alg. 4 on the full grid: solve (L_h - kappa) V = R (R in the padded interior
// layout, consumed).  FP64: in place, *V = R.  FP32 with refinement: an FP32
// solve (FP32 column transforms around the FP64 row solves) of R into A, then
// per refine step: R <- R - (L_h - kappa) d for the last correction d (FP64),
// and the FP32 solve of R as the next correction; *V = A, the sum of them.
kfbi_status grid_solve(kfbi_prob* p, const double** V) {
    hipStream_t s = p->ctx->stream;
    const double inv = 2.0 / p->N;
    if (p->precision == KFBI_FP64) {
        HIP_TRY(launch_dst_cols(p->dp, p->R, p->R, 1.0, false, p->dstB, s));
        HIP_TRY(launch_rows_solve(p->dp, p->R, s));
        HIP_TRY(launch_dst_cols(p->dp, p->R, p->R, inv, false, p->dstB, s));
        *V = p->R;
        return KFBI_OK;
    }
    // corrections: the first lands in A; middle ones in D (then added to A while
    // forming the next residual); the last is accumulated into A directly
    for (int k = 0; k <= p->refine; ++k) {
        if (k == 1) HIP_TRY(launch_residual(p->dp, p->A, p->R, nullptr, s));
        if (k >= 2) HIP_TRY(launch_residual(p->dp, p->D, p->R, p->A, s));
        HIP_TRY(launch_dst_cols_f32(p->dp, p->R, p->X32, 1.0, p->dstB, s));
        HIP_TRY(launch_rows_solve_f32(p->dp, p->X32, s));
        const bool middle = k > 0 && k < p->refine;
        HIP_TRY(launch_dst_cols_f32_to64(p->dp, p->X32, middle ? p->D : p->A, inv, k > 0 && !middle, p->dstB, s));
    }
    *V = p->A;
    return KFBI_OK;
}

// Dense interface solve: R <- f~ (+ corrections), the grid solve, then
// interpolation at the samples (v+ into vz, d_n v+ into dnz; either may be
// null) and, optionally, the grid written to `vgrid`.  normal_jump: the
// density in js is [d_n v] (else [v]).
kfbi_status dense_interface_solve(kfbi_prob* p, bool normal_jump, JumpSrc js, const double* f, bool mask,
                                  double* vgrid, bool mask_out, double* vz, double* dnz = nullptr) {
    hipStream_t s = p->ctx->stream;
    if (js.phi) {
        HIP_TRY(launch_spline(p->dp, js.phi, p->s2a, nullptr, s));
        js.phi_s2 = p->s2a;
    }
    if (js.fgam) {
        HIP_TRY(launch_spline(p->dp, js.fgam, p->s2b, nullptr, s));
        js.fgam_s2 = p->s2b;
    }
    const DevPlan dv = plan_view(p, normal_jump, false);
    HIP_TRY(launch_fill_rhs(dv, f, mask, p->R, s));
    HIP_TRY(launch_correct(dv, js, nullptr, nullptr, p->R, nullptr, s));
    const double* V = nullptr;
    if (kfbi_status e = grid_solve(p, &V)) return e;
    if (vz) HIP_TRY(launch_interp_grid(dv, js, V, vz, s));
    if (dnz) HIP_TRY(launch_interp_grid(plan_view(p, normal_jump, true), js, V, dnz, s));
    if (vgrid) HIP_TRY(launch_grid_out(dv, V, mask_out, vgrid, s));
    return KFBI_OK;
}

// K_D phi or K_N phi (op) without the dense grid (correction, sparse fast
// solve, reduction and interpolation).  With corr_ready the corrections are
// already in corr_il (made by the previous GMRES step's emit launch) and the
// correction launch is skipped.
kfbi_status sparse_apply(kfbi_prob* p, int op, const double* phi, const double* phi_s2, double* out, const int* skip,
                         const GmresBufs* gm, hipStream_t s, bool corr_ready = false) {
    JumpSrc js{phi, phi_s2, nullptr, nullptr, nullptr, nullptr};
    const DevPlan d = op_view(p, op);
    hipEvent_t* ev = nullptr;
    if (p->timing && p->t_count < kfbi_prob::kMaxTimed && !graph_rec()) {
        if (p->ev.empty()) {
            p->ev.assign(6 * kfbi_prob::kMaxTimed, nullptr);
            for (auto& e : p->ev) HIP_TRY(hipEventCreate(&e));
        }
        ev = &p->ev[6 * p->t_count++];
    }
    // each stage is one kernel launch; with timing on, the launch records its
    // own start and end events
    auto stage = [&](int q) {
        if (ev) launch_events() = LaunchEvents{ev[2 * q], ev[2 * q + 1]};
    };
    stage(0);
    if (!corr_ready) HIP_TRY(launch_correct(d, js, nullptr, p->corr_il, nullptr, skip, s));
    if (ev && launch_events().start) {            // nothing was launched
        launch_events() = LaunchEvents{};
        HIP_TRY(hipEventRecord(ev[0], s));
        HIP_TRY(hipEventRecord(ev[1], s));
    }
    stage(1);
    HIP_TRY(launch_modes(d, p->corr_il, p->partial, p->Rm, skip, s));
    stage(2);
    HIP_TRY(launch_reduce_interp(d, js, p->partial, p->G, out, skip, gm, s));
    launch_events() = LaunchEvents{};
    return KFBI_OK;
}

// K_D phi or K_N phi (op) of a caller's density, checked first: the apply's
// launches skip when the check finds a NaN or Inf, so nothing is written, and
// the call waits for the check's flag.
kfbi_status checked_apply(kfbi_prob* p, int op, const double* phi, double* out) {
    hipStream_t s = p->ctx->stream;
    HIP_TRY(launch_nonfinite(p->M, phi, p->d_flag, s));
    HIP_TRY(launch_spline(p->dp, phi, p->s2a, p->d_flag, s));
    if (kfbi_status e = sparse_apply(p, op, phi, p->s2a, out, p->d_flag, nullptr, s)) return e;
    HIP_TRY(hipMemcpyAsync(&p->h_flag, p->d_flag, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (p->h_flag) return set_err(KFBI_ERR_NONFINITE, "NaN or Inf in the density");
    return KFBI_OK;
}

// Restarted GMRES on K_D phi = ghat (ghat already in p->gm.ghat).  Steps are
// enqueued in batches; with tol > 0 the host polls the device state after each
// batch, with tol <= 0 the work is fixed and the host waits once at the end.
// One GMRES step is the apply and the orthogonalisation.  Outside timing mode
// each step's emit launch also makes the next apply's corrections, so the
// apply starts from them; run_gmres makes the first step's.  With timing on the
// corrections get their own launch, timed as a stage of the apply.
kfbi_status enqueue_steps(kfbi_prob* p, int op, int nsteps, hipStream_t s) {
    GmresBufs b = p->gm;
    const int* skip = &b.st->converged;
    const bool fused = !p->timing;
    for (int k = 0; k < nsteps; ++k) {
        if (kfbi_status e = sparse_apply(p, op, b.xcur, b.s2cur, b.w, skip, &p->gm, s, fused)) return e;
        if (fused) {
            HIP_TRY(launch_gmres_step_corr(op_view(p, op), b, p->corr_il, s));
        } else {
            HIP_TRY(launch_gmres_step(p->dp.taps, p->dp.M, b, s));
        }
    }
    return KFBI_OK;
}

// Record kGraphSteps >> k GMRES steps into a graph once per problem.  All
// launch arguments are fixed device pointers and the steps read their
// parameters from the device state, so one graph serves every call.  If
// recording is not possible the steps are launched directly.
void ensure_graph(kfbi_prob* p, int op, int k) {
    if (p->gexec[op][k] || p->graph_failed[op][k]) return;
    const bool timing = p->timing;
    p->timing = false;
    p->graph_failed[op][k] = !record_graph(p->ctx->stream, &p->gexec[op][k], [&](hipStream_t s) {
        return enqueue_steps(p, op, kfbi_prob::kGraphSteps >> k, s);
    });
    p->timing = timing;
}

// One restarted-GMRES run in flight on a problem's stream (run_gmres and
// run_gmres_pair drive it).
struct GmresRun {
    kfbi_prob* p = nullptr;
    int op = kOpD;
    int max_steps = 0, steps = 0, batches = 0;
    bool use_graph = false, poll_each = true, extended = false, finished = false;
};

// Set up GMRES on K phi = ghat (K_D or K_N by op) from phi_in: ghat <- rhs
// (null: already in p->gm.ghat), the state, and the first K input with its
// spline and corrections, in two launches (gm_start); xout (may be null)
// receives the final iterate from the device.  The run takes at most max_iter
// Arnoldi steps and one residual step per cycle end: those step slots are
// launched.  A nonzero guess takes one residual step more, at the start; the
// run finds that in its last poll and launches one more slot (gmres_more).
kfbi_status gmres_start(kfbi_prob* p, int op, const double* rhs, const double* phi_in, double tol, int max_iter,
                        double* xout, GmresRun* r) {
    hipStream_t s = p->ctx->stream;
    const DevPlan d = op_view(p, op);
    HIP_TRY(launch_gmres_start(&d, p->dp.taps, p->M, p->gm, rhs, phi_in, tol, max_iter, p->reorth, xout,
                               p->timing ? nullptr : p->corr_il, s));
    const int m = std::max(1, p->restart);
    *r = GmresRun{};
    r->p = p;
    r->op = op;
    r->max_steps = max_iter + (max_iter + m - 1) / m;
    r->use_graph = !p->timing;
    r->poll_each = tol > 0;
    if (r->use_graph)                                   // recorded at the first run, not inside a later one
        for (int k = 0; k < kfbi_prob::kGraphSizes; ++k) ensure_graph(p, op, k);
    return KFBI_OK;
}

// After the poll of the last slot: whether the run still needs its one extra
// residual step (a nonzero initial guess); if so the slot is added.
bool gmres_more(GmresRun& r) {
    if (r.p->st_host.converged || r.extended) return false;
    r.extended = true;
    r.max_steps += 1;
    return true;
}

// Enqueue the next batch of steps: kGraphSteps, or the largest power of two
// not above what is left (a replayed graph unless per-launch timing is on);
// returns through *poll whether the state should be read after it (every
// batch when the run can stop early, else only after the last).  A run that
// can stop early takes batches of 8, 16, then 32 steps: the steps launched
// after the device has converged return at once but still cost their
// launches (about 7 us a step), a poll costs about three of them.
kfbi_status gmres_batch(GmresRun& r, bool* poll) {
    kfbi_prob* p = r.p;
    hipStream_t s = p->ctx->stream;
    const int cap = r.poll_each ? std::min(kfbi_prob::kGraphSteps, 8 << std::min(r.batches, 4)) : kfbi_prob::kGraphSteps;
    const int want = std::min(r.max_steps - r.steps, cap);
    int k = 0;
    while ((kfbi_prob::kGraphSteps >> k) > want && k + 1 < kfbi_prob::kGraphSizes) ++k;
    const int n = kfbi_prob::kGraphSteps >> k;
    if (r.use_graph) ensure_graph(p, r.op, k);
    if (r.use_graph && p->gexec[r.op][k]) {
        HIP_TRY(hipGraphLaunch(p->gexec[r.op][k], s));
    } else if (kfbi_status e = enqueue_steps(p, r.op, n, s)) {
        return e;
    }
    r.steps += n;
    r.batches += 1;
    *poll = r.poll_each || r.steps >= r.max_steps;
    return KFBI_OK;
}

// Wait for the stream and take the state the device last published (every
// residual step, a run's end and its start publish it) into p->st_host.
kfbi_status gmres_read_state(kfbi_prob* p) {
    HIP_TRY(hipStreamSynchronize(p->ctx->stream));
    p->st_host = *p->st_pub;
    return KFBI_OK;
}

// Restarted GMRES on K phi = ghat (K_D or K_N by op; ghat <- rhs, or already
// in p->gm.ghat when rhs is null).  Steps go in batches (a replayed graph
// unless per-launch timing is on); with tol > 0 the host polls the device
// state after each batch, with tol <= 0 the work is fixed and the host waits
// once at the end.
kfbi_status run_gmres(kfbi_prob* p, int op, const double* rhs, const double* phi_in, double tol, int max_iter,
                      GmresState* out, double* x_out = nullptr) {
    GmresRun r;
    if (kfbi_status e = gmres_start(p, op, rhs, phi_in, tol, max_iter, x_out, &r)) return e;
    for (;;) {
        if (r.steps >= r.max_steps && !gmres_more(r)) break;
        bool poll = false;
        if (kfbi_status e = gmres_batch(r, &poll)) return e;
        if (poll) {
            if (kfbi_status e = gmres_read_state(p)) return e;
            if (p->st_host.converged) break;
        }
    }
    *out = p->st_host;
    return KFBI_OK;
}

// GMRES on two problems at once, each on its own stream: every round enqueues a
// batch on each problem that is still running, then reads both states, so the
// two runs overlap on the device.
kfbi_status run_gmres_pair(kfbi_prob* pa, int opa, const double* xa, kfbi_prob* pb, int opb, const double* xb,
                           GmresState* outa, GmresState* outb) {
    GmresRun r[2];
    if (kfbi_status e = gmres_start(pa, opa, nullptr, xa, pa->tol, pa->max_iter, nullptr, &r[0])) return e;
    if (kfbi_status e = gmres_start(pb, opb, nullptr, xb, pb->tol, pb->max_iter, nullptr, &r[1])) return e;
    while (!(r[0].finished && r[1].finished)) {
        for (auto& q : r) {
            if (q.finished) continue;
            bool poll = false;
            if (kfbi_status e = gmres_batch(q, &poll)) return e;
        }
        for (auto& q : r) {
            if (q.finished) continue;
            if (kfbi_status e = gmres_read_state(q.p)) return e;
            if (q.p->st_host.converged || (q.steps >= q.max_steps && !gmres_more(q))) q.finished = true;
        }
    }
    *outa = pa->st_host;
    *outb = pb->st_host;
    return KFBI_OK;
}

// GMRES on K x = rhs for the operator op, from the initial guess in x.
kfbi_status gmres_call(kfbi_prob* p, int op, const double* rhs, double* x, double tol, int max_iter, int* iters,
                       int* applies, double* rel_res) {
    if (!p) return set_err(KFBI_ERR_ARG, "prob is NULL");
    if (kfbi_status e = check_ptr(rhs, "rhs")) return e;
    if (kfbi_status e = check_ptr(x, "x")) return e;
    if (max_iter <= 0) return set_err(KFBI_ERR_ARG, "max_iter must be positive");
    HIP_TRY(hipSetDevice(p->ctx->device));
    GmresState st{};
    if (kfbi_status e = run_gmres(p, op, rhs, x, tol, max_iter, &st, x)) return e;
    if (st.converged == kGmNonfinite) return set_err(KFBI_ERR_NONFINITE, "NaN or Inf in rhs or the initial guess");
    if (iters) *iters = st.it;
    if (applies) *applies = st.it + st.res_applies;
    if (rel_res) *rel_res = st.relres;
    if (st.converged == 1) return KFBI_OK;
    return set_err(KFBI_NOT_CONVERGED, "GMRES reached the iteration cap");
}

// ---------------------------------------------------------------- Richardson and BiCGSTAB

enum IterMethod { kRich = 0, kBicg = 1 };
constexpr int kIterBatch[2] = {8, 4};   // iterations per replayed batch (8 applies each)

// One K_D apply of `in` into ib.w (spline, correction, sparse solve, reduction),
// skipped once the run is done.
kfbi_status iter_apply(kfbi_prob* p, const double* in, const int* skip, hipStream_t s) {
    HIP_TRY(launch_spline(p->dp, in, p->ib.s2, skip, s));
    return sparse_apply(p, kOpD, in, p->ib.s2, p->ib.w, skip, nullptr, s);
}

kfbi_status enqueue_iters(kfbi_prob* p, int method, int n, hipStream_t s) {
    const IterBufs& B = p->ib;
    const int* skip = &B.st->done;
    for (int k = 0; k < n; ++k) {
        if (method == kRich) {
            if (kfbi_status e = iter_apply(p, B.x, skip, s)) return e;
            HIP_TRY(launch_iter_step(kIterRich, B, s));
        } else {
            if (kfbi_status e = iter_apply(p, B.q, skip, s)) return e;
            HIP_TRY(launch_iter_step(kIterBicgHalf, B, s));
            if (kfbi_status e = iter_apply(p, B.q, skip, s)) return e;
            HIP_TRY(launch_iter_step(kIterBicgFull, B, s));
        }
    }
    return KFBI_OK;
}

// Richardson (x <- x + gamma (b - K_D x)) or BiCGSTAB on K_D x = rhs from the
// initial guess in x; same stopping rule as GMRES (relative to the initial
// residual).  Batches of iterations are replayed from a graph; the host polls
// the device state between batches.
kfbi_status run_iters(kfbi_prob* p, int method, const double* rhs, double* x, double gamma, double tol, int max_iter,
                      IterState* out) {
    if (!p) return set_err(KFBI_ERR_ARG, "prob is NULL");
    if (kfbi_status e = check_ptr(rhs, "rhs")) return e;
    if (kfbi_status e = check_ptr(x, "x")) return e;
    if (max_iter <= 0) return set_err(KFBI_ERR_ARG, "max_iter must be positive");
    HIP_TRY(hipSetDevice(p->ctx->device));
    hipStream_t s = p->ctx->stream;
    const IterBufs& B = p->ib;
    const int M = p->M;
    const bool timing = p->timing;
    p->timing = false;                      // the per-stage events belong to GMRES steps
    struct Restore {
        kfbi_prob* p;
        bool t;
        ~Restore() { p->timing = t; }
    } restore{p, timing};
    HIP_TRY(hipMemcpyAsync(B.b, rhs, M * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(B.x, x, M * sizeof(double), hipMemcpyDeviceToDevice, s));
    static thread_local IterState st0;
    st0 = IterState{};
    st0.max_iter = max_iter;
    st0.tol = tol;
    st0.gamma = gamma;
    HIP_TRY(hipMemcpyAsync(B.st, &st0, sizeof st0, hipMemcpyHostToDevice, s));
    if (method == kBicg) {                  // r0 = b - K x0, r^ = p = r0
        if (kfbi_status e = iter_apply(p, B.x, &B.st->done, s)) return e;
        HIP_TRY(launch_iter_step(kIterBicgInit, B, s));
    }
    if (!p->iexec[method] && !p->iexec_failed[method])
        p->iexec_failed[method] = !record_graph(s, &p->iexec[method], [&](hipStream_t gs) {
            return enqueue_iters(p, method, kIterBatch[method], gs);
        });
    const int nb = kIterBatch[method];
    const int batches = (max_iter + 1) / nb + 2;
    IterState st{};
    for (int b = 0; b < batches; ++b) {
        if (p->iexec[method]) {
            HIP_TRY(hipGraphLaunch(p->iexec[method], s));
        } else if (kfbi_status e = enqueue_iters(p, method, nb, s)) {
            return e;
        }
        HIP_TRY(hipMemcpyAsync(&st0, B.st, sizeof st0, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        st = st0;
        if (st.done) break;
    }
    if (st.done == kIterNonfinite) return set_err(KFBI_ERR_NONFINITE, "NaN or Inf in rhs or the initial guess");
    if (method == kBicg) {                  // the true residual of the final iterate
        if (kfbi_status e = iter_apply(p, B.x, nullptr, s)) return e;
        HIP_TRY(launch_iter_step(kIterTrueRes, B, s));
        HIP_TRY(hipMemcpyAsync(&st0, B.st, sizeof st0, hipMemcpyDeviceToHost, s));
    }
    HIP_TRY(hipMemcpyAsync(x, B.x, M * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    *out = st0;
    return KFBI_OK;
}

// ---------------------------------------------------------------- the Neumann solve in parts

kfbi_status neumann_check(kfbi_prob* p, const NeumannIO& io) {
    if (!p) return set_err(KFBI_ERR_ARG, "prob is NULL");
    for (auto [ptr, name] : {std::pair<const void*, const char*>{io.f_grid, "f_grid"}, {io.f_gamma, "f_gamma"},
                             {io.g_n, "g_n"}, {io.u_grid, "u_grid"}, {io.u_gamma, "u_gamma"},
                             {io.dn_gamma, "dn_gamma"}, {io.psi, "psi"}})
        if (kfbi_status s = check_ptr(ptr, name)) return s;
    if (!(p->kappa > 0.0)) return set_err(KFBI_ERR_ARG, "the Neumann problem needs kappa > 0");
    return KFBI_OK;
}

// g^ = g_n - d_n (Y f)^+ into the GMRES right-hand side.
kfbi_status neumann_prepare(kfbi_prob* p, const NeumannIO& io) {
    JumpSrc jy{nullptr, nullptr, io.f_gamma, nullptr, nullptr, nullptr};
    if (kfbi_status e = dense_interface_solve(p, true, jy, io.f_grid, true, nullptr, false, nullptr, p->tmpM)) return e;
    HIP_TRY(launch_axpby(p->M, 1.0, io.g_n, -1.0, p->tmpM, p->gm.ghat, p->ctx->stream));
    return KFBI_OK;
}

// u = v_psi + Y f with its trace and normal derivative, and psi out.
kfbi_status neumann_finish(kfbi_prob* p, const NeumannIO& io) {
    JumpSrc jf{p->gm.phi, nullptr, io.f_gamma, nullptr, nullptr, nullptr};
    if (kfbi_status e = dense_interface_solve(p, true, jf, io.f_grid, true, io.u_grid, true, io.u_gamma, io.dn_gamma))
        return e;
    HIP_TRY(hipMemcpyAsync(io.psi, p->gm.phi, p->M * sizeof(double), hipMemcpyDeviceToDevice, p->ctx->stream));
    return KFBI_OK;
}

}  // namespace

namespace kfbi {

kfbi_status solve_neumann_pair(kfbi_prob* pa, const NeumannIO& ia, kfbi_prob* pb, const NeumannIO& ib, int* iters_a,
                               int* iters_b) {
    if (kfbi_status e = neumann_check(pa, ia)) return e;
    if (kfbi_status e = neumann_check(pb, ib)) return e;
    HIP_TRY(hipSetDevice(pa->ctx->device));
    if (kfbi_status e = neumann_prepare(pa, ia)) return e;
    if (kfbi_status e = neumann_prepare(pb, ib)) return e;
    GmresState sa{}, sb{};
    if (kfbi_status e = run_gmres_pair(pa, kOpN, ia.psi, pb, kOpN, ib.psi, &sa, &sb)) return e;
    if (sa.converged == kGmNonfinite || sb.converged == kGmNonfinite)
        return set_err(KFBI_ERR_NONFINITE, "NaN or Inf in f, f_gamma, g_n or psi");
    if (kfbi_status e = neumann_finish(pa, ia)) return e;
    if (kfbi_status e = neumann_finish(pb, ib)) return e;
    if (iters_a) *iters_a = sa.it;
    if (iters_b) *iters_b = sb.it;
    if (sa.converged == 1 && sb.converged == 1) return KFBI_OK;
    return set_err(KFBI_NOT_CONVERGED, "GMRES reached the iteration cap");
}

}  // namespace kfbi

extern "C" {

const char* kfbi_status_str(kfbi_status s) {
    switch (s) {
        case KFBI_OK: return "ok";
        case KFBI_NOT_CONVERGED: return "not converged";
        case KFBI_ERR_ARG: return "invalid argument";
        case KFBI_ERR_GEOMETRY: return "unsupported geometry";
        case KFBI_ERR_OOM: return "out of device memory";
        case KFBI_ERR_DEVICE: return "device error";
        case KFBI_ERR_BUDGET: return "over memory budget";
        case KFBI_ERR_NONFINITE: return "non-finite data";
        case KFBI_ERR_UNSUPPORTED: return "unsupported configuration";
        default: return "unknown status";
    }
}

const char* kfbi_last_error(void) { return last_error().c_str(); }

kfbi_status kfbi_ctx_create(int device, void* hip_stream, kfbi_ctx** out) {
    if (!out) return set_err(KFBI_ERR_ARG, "out is NULL");
    int count = 0;
    HIP_TRY(hipGetDeviceCount(&count));
    if (device < 0 || device >= count) return set_err(KFBI_ERR_ARG, "no such device");
    HIP_TRY(hipSetDevice(device));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, device));
    kfbi_ctx* c = new (std::nothrow) kfbi_ctx;
    if (!c) return set_err(KFBI_ERR_ARG, "host allocation failed");
    c->device = device;
    c->lds_max = prop.sharedMemPerBlock;
    c->num_cu = prop.multiProcessorCount;
    // the no-alloc scratch's address on this device, resolved here once; a
    // failure only matters to kfbi_apply_noalloc, which reports it (and retries)
    void* scr = nullptr;
    if (scratch_on(device, &scr) != KFBI_OK) last_error().clear();
    if (hip_stream) {
        c->stream = static_cast<hipStream_t>(hip_stream);
    } else {
        hipError_t e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            delete c;
            return set_err(KFBI_ERR_DEVICE, hipGetErrorString(e));
        }
        c->own_stream = true;
    }
    *out = c;
    return KFBI_OK;
}

kfbi_status kfbi_ctx_destroy(kfbi_ctx* ctx) {
    if (!ctx) return KFBI_OK;
    if (ctx->own_stream) hipStreamDestroy(ctx->stream);
    delete ctx;
    return KFBI_OK;
}

kfbi_status kfbi_ctx_sync(kfbi_ctx* ctx) {
    if (!ctx) return set_err(KFBI_ERR_ARG, "ctx is NULL");
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return KFBI_OK;
}

kfbi_status kfbi_prob_create(kfbi_ctx* ctx, const kfbi_desc* d, kfbi_prob** out) {
    if (!ctx || !d || !out || !d->xy) return set_err(KFBI_ERR_ARG, "NULL argument");
    const int n = d->n;
    if (n < 64 || n > 4096 || (n & (n - 1))) return set_err(KFBI_ERR_UNSUPPORTED, "n must be a power of two in [64, 4096]");
    if (d->m < 3 || d->m > kMaxSamples) return set_err(KFBI_ERR_ARG, "m must be in [3, 12288]");
    if (!(d->hi > d->lo) || !std::isfinite(d->lo) || !std::isfinite(d->hi)) return set_err(KFBI_ERR_ARG, "bad box");
    if (!(d->kappa >= 0.0) || !std::isfinite(d->kappa)) return set_err(KFBI_ERR_ARG, "kappa must be finite and >= 0");
    if (d->precision != KFBI_FP64 && d->precision != KFBI_FP32_REFINED)
        return set_err(KFBI_ERR_ARG, "precision must be KFBI_FP64 or KFBI_FP32_REFINED");
    if (d->precision == KFBI_FP32_REFINED && d->refine_steps > 4)
        return set_err(KFBI_ERR_ARG, "refine_steps must be at most 4");
    HIP_TRY(hipSetDevice(ctx->device));
    kfbi_prob* p = new (std::nothrow) kfbi_prob;
    if (!p) return set_err(KFBI_ERR_ARG, "host allocation failed");
    p->ctx = ctx;
    try {
        p->plan = build_plan(d->xy, d->m, n, d->lo, d->hi);
    } catch (const GeometryError& ge) {
        delete p;
        return set_err(KFBI_ERR_GEOMETRY, ge.msg);
    } catch (const std::bad_alloc&) {
        delete p;
        return set_err(KFBI_ERR_ARG, "host allocation failed");
    }
    const Plan& P = p->plan;
    p->kappa = d->kappa;
    p->tol = d->tol > 0 ? d->tol : 1e-10;
    p->restart = d->restart > 0 ? std::min(d->restart, kMaxRestart) : 50;
    p->max_iter = d->max_iter > 0 ? d->max_iter : 500;
    p->precision = d->precision;
    p->refine = d->precision == KFBI_FP32_REFINED ? (d->refine_steps < 0 ? 1 : d->refine_steps) : 0;
    p->N = n;
    p->n = n - 1;
    p->M = d->m;
    p->Q = (int)P.q_axis.size();
    p->I = (int)P.irr_i.size();
    if (p->M > kMaxSamples) {
        delete p;
        return set_err(KFBI_ERR_UNSUPPORTED, "more than " + std::to_string(kMaxSamples) + " samples");
    }
    // modes per workgroup of the sparse fast solve: the most the LDS holds that
    // still leaves a workgroup for at least half of the compute units
    {
        int rmax = 0;
        for (int r = kMaxModesPerGroup; r >= 1 && !rmax; r /= 2)
            if (modes_lds_bytes(n, r) <= ctx->lds_max) rmax = r;
        if (!rmax) {
            delete p;
            return set_err(KFBI_ERR_UNSUPPORTED, "problem too large for the local data share");
        }
        p->Rm = 1;
        for (int r = rmax; r >= 1; r /= 2)
            if ((p->n + r - 1) / r >= ctx->num_cu / 2 || r == 1) {
                p->Rm = r;
                break;
            }
        p->G = (p->n + p->Rm - 1) / p->Rm;
        // the autotuner may halve Rm once: room for that many partial rows
        p->Gcap = (p->n + std::max(1, p->Rm / 2) - 1) / std::max(1, p->Rm / 2);
    }
    p->dstB = dst_default_tile(n, cpx_bytes(p->precision), ctx->lds_max, n, ctx->num_cu);
    if (p->dstB == 0) {
        delete p;
        return set_err(KFBI_ERR_UNSUPPORTED, "grid too large for the column transforms' local data share");
    }

    kfbi_status st = KFBI_OK;
    auto fail = [&](kfbi_status s) {
        free_prob(p);
        delete p;
        return s;
    };
    DevPlan& dp = p->dp;
    dp.n = p->n;
    dp.N = n;
    dp.M = p->M;
    dp.Q = p->Q;
    dp.I = p->I;
    dp.log2N = 0;
    while ((1 << dp.log2N) < n) dp.log2N++;
    dp.lo = P.lo;
    dp.h = P.h;
    dp.h2 = P.h * P.h;
    dp.inv_h2 = 1.0 / (P.h * P.h);
    dp.kappa = p->kappa;
    std::vector<int> sxy(p->M);
    for (int k = 0; k < p->M; ++k) sxy[k] = (P.cp_sx[k] > 0 ? 1 : 0) | (P.cp_sy[k] > 0 ? 2 : 0);
    std::vector<double> sinq(n / 2 + 1);
    for (int k = 0; k <= n / 2; ++k) sinq[k] = std::sin(M_PI * k / n);
    sinq[n / 2] = 1.0;
    const int K = 30;
    dp.K = K;
    std::vector<int> colptr(P.col_ptr.begin(), P.col_ptr.end());
    // node table of the sparse sine sums: kModeWaves sub-tables of 64 lanes
    // (512 workers).  A column's nodes form one piece, or several pieces of at
    // most `cap` nodes when the column is long (its extra pieces' sums are added
    // to the first piece's in a fixed order); pieces go largest first to the
    // least loaded worker, each worker's pieces in order, and sub-table w's rows
    // are the longest worker list among its lanes
    std::vector<int> sub_off(kModeWaves + 1, 0), il_ij, il_pos(std::max(p->I, 1), 0), split;
    {
        constexpr int NW = kModeWaves * 64;
        auto xpos_of = [&](int i) { return i + (i - 1) / (n / 64); };
        int cap = std::max(1, (p->I + NW - 1) / NW);
        for (;;) {
            long extra = 0;
            for (int i = 0; i <= n; ++i) extra += std::max(0, (colptr[i + 1] - colptr[i] + cap - 1) / cap - 1);
            if (extra <= kMaxExtra) break;
            cap *= 2;
        }
        struct Piece {
            int first, count, dest;
        };
        std::vector<Piece> pieces;
        int n_extra = 0;
        for (int i = 0; i <= n; ++i) {
            const int cnt = colptr[i + 1] - colptr[i];
            if (cnt == 0) continue;
            const int np = (cnt + cap - 1) / cap;
            if (np > 1) {
                split.push_back(xpos_of(i));
                split.push_back(n_extra);
                split.push_back(np - 1);
            }
            for (int k = 0; k < np; ++k) {
                const int a = colptr[i] + k * cap, b = std::min(colptr[i + 1], a + cap);
                pieces.push_back({a, b - a, k == 0 ? xpos_of(i) : (kExtraFlag | n_extra++)});
            }
        }
        std::vector<int> order(pieces.size());
        for (size_t k = 0; k < order.size(); ++k) order[k] = (int)k;
        std::stable_sort(order.begin(), order.end(),
                         [&](int a, int b) { return pieces[a].count > pieces[b].count; });
        using Load = std::pair<int, int>;               // (nodes so far, worker)
        std::priority_queue<Load, std::vector<Load>, std::greater<Load>> heap;
        for (int w = 0; w < NW; ++w) heap.push({0, w});
        std::vector<std::vector<int>> wpieces(NW);
        std::vector<int> load(NW, 0);
        for (int k : order) {
            const Load top = heap.top();
            heap.pop();
            wpieces[top.second].push_back(k);
            load[top.second] += pieces[k].count;
            heap.push({load[top.second], top.second});
        }
        for (int w = 0; w < kModeWaves; ++w) {
            int t = 0;
            for (int L = 0; L < 64; ++L) t = std::max(t, load[w * 64 + L]);
            sub_off[w + 1] = sub_off[w] + (t + kSlots - 1) / kSlots * kSlots;
        }
        const int T = std::max(sub_off[kModeWaves], kSlots);
        dp.T = T;
        il_ij.assign((size_t)T * 64, 0);
        for (int w = 0; w < NW; ++w) {
            const int sub = w / 64, L = w % 64;
            int t = sub_off[sub];
            for (int k : wpieces[w]) {
                const Piece& pc = pieces[k];
                for (int r = pc.first; r < pc.first + pc.count; ++r, ++t) {
                    const size_t slot = (size_t)t * 64 + L;
                    const bool last = r + 1 == pc.first + pc.count;
                    il_ij[slot] = (last ? (int)0x80000000u : 0) | (pc.dest << 16) | P.irr_j[r];
                    il_pos[r] = (int)slot;
                }
            }
        }
        dp.n_split = (int)split.size() / 3;
    }
    std::vector<int4> cpk(p->M);
    for (int k = 0; k < p->M; ++k) cpk[k] = make_int4(P.cp_i0[k], P.cp_j0[k], sxy[k], 0);
    // correction chunks: irregular nodes in the order of their first crossing
    // along Gamma, cut where a chunk would exceed kCorrChunk nodes or its
    // crossings' segments (with the spline filter's reach) a window of
    // kCorrWindow knots
    std::vector<int> cc_node(std::max(p->I, 1), 0);
    std::vector<int4> cc_chunk;
    {
        const int M = p->M, I = p->I, reach = K + 1;
        std::vector<int> key(I);
        for (int r = 0; r < I; ++r) {
            cc_node[r] = r;
            key[r] = P.q_geo[P.arm_q[4 * r]].seg;
        }
        std::stable_sort(cc_node.begin(), cc_node.begin() + I, [&](int a, int b) { return key[a] < key[b]; });
        auto offset = [M](int seg, int ref) {        // seg - ref on the circle, in (-M/2, M/2]
            int o = ((seg - ref) % M + M) % M;
            return o > M / 2 ? o - M : o;
        };
        int first = 0;
        while (first < I) {
            const int ref = key[cc_node[first]];
            int lo = 0, hi = 0, end = first;
            while (end < I && end - first < kCorrChunk) {
                const int r = cc_node[end];
                int nlo = lo, nhi = hi;
                for (int a = 0; a < 4 && P.arm_q[4 * r + a] >= 0; ++a) {
                    const int o = offset(P.q_geo[P.arm_q[4 * r + a]].seg, ref);
                    nlo = std::min(nlo, o);
                    nhi = std::max(nhi, o + 1);           // the segment's end knot
                }
                if (end > first && (nhi - nlo + 1) + 2 * reach > kCorrWindow) break;
                lo = nlo;
                hi = nhi;
                ++end;
            }
            const int width = (hi - lo + 1) + 2 * reach;
            if (width > kCorrWindow) return fail(set_err(KFBI_ERR_GEOMETRY, "an irregular node's crossings lie too far apart along the curve"));
            const int k0 = ((ref + lo - reach) % M + M) % M;
            cc_chunk.push_back(make_int4(first, end, k0, width));
            first = end;
        }
        dp.n_cc = (int)cc_chunk.size();
    }
    if (cc_chunk.empty()) cc_chunk.push_back(make_int4(0, 0, 0, 0));
    // the nodes' data by chunk, kCorrChunk places per chunk (pads have no arms),
    // so that a workgroup finds its chunk's data without reading the chunk first
    const size_t n_places = cc_chunk.size() * (size_t)kCorrChunk;
    std::vector<int4> cc_arm(n_places, make_int4(-1, -1, -1, -1));
    std::vector<double4> cc_d(n_places, make_double4(0, 0, 0, 0));
    std::vector<double> cc_s(n_places, 0.0);
    std::vector<int> cc_pos(n_places, 0);
    for (int c = 0; c < dp.n_cc; ++c) {
        const int4 ch = cc_chunk[c];
        for (int at = ch.x; at < ch.y; ++at) {
            const int r = cc_node[at];
            const size_t q = (size_t)c * kCorrChunk + (at - ch.x);
            cc_arm[q] = make_int4(P.arm_q[4 * r], P.arm_q[4 * r + 1], P.arm_q[4 * r + 2], P.arm_q[4 * r + 3]);
            cc_d[q] = make_double4(P.arm_d[4 * r], P.arm_d[4 * r + 1], P.arm_d[4 * r + 2], P.arm_d[4 * r + 3]);
            cc_s[q] = P.irr_s[r];
            cc_pos[q] = il_pos[r];
        }
    }
    if ((st = upload(p, &dp.cc_arm, cc_arm)) || (st = upload(p, &dp.cc_d, cc_d)) || (st = upload(p, &dp.cc_s, cc_s)) ||
        (st = upload(p, &dp.cc_pos, cc_pos)) || (st = upload(p, &dp.cc_chunk, cc_chunk)))
        return fail(st);
    if ((st = upload(p, &dp.q_geo, P.q_geo)) || (st = upload(p, &dp.q_axis, P.q_axis)) ||
        (st = upload(p, &dp.z_geo, P.z_geo)) || (st = upload(p, &dp.zx, P.px)) || (st = upload(p, &dp.zy, P.py)) ||
        (st = upload(p, &dp.irr_i, P.irr_i)) || (st = upload(p, &dp.irr_j, P.irr_j)) ||
        (st = upload(p, &dp.irr_s, P.irr_s)) || (st = upload(p, &dp.arm_q, P.arm_q)) ||
        (st = upload(p, &dp.arm_d, P.arm_d)) || (st = upload(p, &dp.col_ptr, colptr)) ||
        (st = upload(p, &dp.sub_off, sub_off)) || (st = upload(p, &dp.split, split)) || (st = upload(p, &dp.il_ij, il_ij)) ||
        (st = upload(p, &dp.il_pos, il_pos)) || (st = upload(p, &dp.cp_pack, cpk)) ||
        (st = upload(p, &dp.cp_i0, P.cp_i0)) || (st = upload(p, &dp.cp_j0, P.cp_j0)) ||
        (st = upload(p, &dp.cp_sxy, sxy)) || (st = upload(p, &dp.cp_w, P.cp_w)) || (st = upload(p, &p->cp_wn, P.cp_wn)) ||
        (st = upload(p, &dp.cp_out, P.cp_out)) || (st = upload(p, &dp.inside, P.inside)) ||
        (st = upload(p, &dp.sinq, sinq)) || (st = upload(p, &dp.modes, mode_constants(n, P.h, p->kappa))) ||
        (st = upload(p, &dp.taps, spline_filter_taps(K))))
        return fail(st);
    for (int w = 0; w <= kModeWaves; ++w) dp.sub_offv[w] = sub_off[w];
    const int M = p->M, m = p->restart;
    if ((st = dev_alloc(p, &p->corr, p->I)) || (st = dev_alloc(p, &p->corr_il, (size_t)dp.T * 64)) || (st = dev_alloc(p, &p->partial, (size_t)p->Gcap * M)) ||
        (st = dev_alloc(p, &p->R, (size_t)n * n)) || (st = dev_alloc(p, &p->A, (size_t)n * n)) ||
        (st = dev_alloc(p, &p->tmpM, M)) || (st = dev_alloc(p, &p->s2a, M)) || (st = dev_alloc(p, &p->s2b, M)) ||
        (st = dev_alloc(p, &p->d_flag, 1)) ||
        (st = dev_alloc(p, &p->gm.s2cur, M)) || (st = dev_alloc(p, &p->gm.V, (size_t)(m + 1) * M)) ||
        (st = dev_alloc(p, &p->gm.H, (size_t)(m + 1) * m)) || (st = dev_alloc(p, &p->gm.cs, m)) ||
        (st = dev_alloc(p, &p->gm.sn, m)) || (st = dev_alloc(p, &p->gm.g, m + 1)) ||
        (st = dev_alloc(p, &p->gm.ghat, M)) || (st = dev_alloc(p, &p->gm.phi, M)) ||
        (st = dev_alloc(p, &p->gm.xcur, M)) || (st = dev_alloc(p, &p->gm.w, M)) ||
        (st = dev_alloc(p, &p->gm.z, M)) || (st = dev_alloc(p, &p->gm.part, gm_part_size(m, gm_chunks(M), gm_chunks64(M)))) ||
        (st = dev_alloc(p, &p->gm.y, m + 1)) || (st = dev_alloc(p, &p->gm.st, 1)) ||
        (st = dev_alloc(p, &p->gm.cnt, 1)))
        return fail(st);
    {
        IterBufs& ib = p->ib;
        double** vecs[] = {&ib.b, &ib.x, &ib.r, &ib.rhat, &ib.p, &ib.v, &ib.s, &ib.q, &ib.w, &ib.s2};
        for (double** v : vecs)
            if ((st = dev_alloc(p, v, M))) return fail(st);
        if ((st = dev_alloc(p, &ib.st, 1))) return fail(st);
        ib.M = M;
    }
    HIP_TRY(hipMemset(p->gm.cnt, 0, sizeof(unsigned)));
    // the state's host mirror: pinned, coherent host memory the device writes to
    if (hipHostMalloc((void**)&p->st_pub, sizeof(GmresState), hipHostMallocMapped | hipHostMallocCoherent) !=
        hipSuccess) {
        hipGetLastError();
        p->st_pub = nullptr;
        return fail(set_err(KFBI_ERR_OOM, "pinned host allocation of the GMRES state mirror failed"));
    }
    *p->st_pub = GmresState{};
    p->gm.pub = p->st_pub;
    if (p->precision == KFBI_FP32_REFINED && (st = dev_alloc(p, &p->X32, (size_t)n * n))) return fail(st);
    if (p->refine >= 2 && (st = dev_alloc(p, &p->D, (size_t)n * n))) return fail(st);
    // pad slots of the interleaved corrections stay zero for the life of the problem
    HIP_TRY(hipMemset(p->corr_il, 0, sizeof(double) * (size_t)dp.T * 64));
    p->gm.m = m;
    p->gm.gc = gm_chunks(M);
    p->gm.gc64 = gm_chunks64(M);
    *out = p;
    return KFBI_OK;
}

kfbi_status kfbi_prob_destroy(kfbi_prob* p) {
    if (!p) return KFBI_OK;
    hipSetDevice(p->ctx->device);
    hipStreamSynchronize(p->ctx->stream);
    free_prob(p);
    delete p;
    return KFBI_OK;
}

kfbi_status kfbi_prob_info(const kfbi_prob* p, int* m, int* q, int* ni, size_t* bytes) {
    if (!p) return set_err(KFBI_ERR_ARG, "prob is NULL");
    if (m) *m = p->M;
    if (q) *q = p->Q;
    if (ni) *ni = p->I;
    if (bytes) *bytes = p->bytes;
    return KFBI_OK;
}

kfbi_status kfbi_prob_mask(const kfbi_prob* p, unsigned char* inside) {
    if (!p || !inside) return set_err(KFBI_ERR_ARG, "NULL argument");
    std::memcpy(inside, p->plan.inside.data(), p->plan.inside.size());
    return KFBI_OK;
}

kfbi_status kfbi_prob_crossings(const kfbi_prob* p, int* axis, int* nodes, double* t, double* xy) {
    if (!p) return set_err(KFBI_ERR_ARG, "prob is NULL");
    const Plan& P = p->plan;
    for (int k = 0; k < p->Q; ++k) {
        if (axis) axis[k] = P.q_axis[k];
        if (nodes)
            for (int c = 0; c < 4; ++c) nodes[4 * k + c] = P.q_nodes[4 * k + c];
        if (t) t[k] = P.q_t[k];
        if (xy) {
            xy[2 * k] = P.q_x[k];
            xy[2 * k + 1] = P.q_y[k];
        }
    }
    return KFBI_OK;
}

kfbi_status kfbi_prob_points(const kfbi_prob* p, double* xy, double* normal) {
    if (!p) return set_err(KFBI_ERR_ARG, "prob is NULL");
    for (int k = 0; k < p->M; ++k) {
        if (xy) {
            xy[2 * k] = p->plan.px[k];
            xy[2 * k + 1] = p->plan.py[k];
        }
        if (normal) {
            normal[2 * k] = p->plan.z_geo[k].nx;
            normal[2 * k + 1] = p->plan.z_geo[k].ny;
        }
    }
    return KFBI_OK;
}

kfbi_status kfbi_prob_irregular(const kfbi_prob* p, int* ij) {
    if (!p || !ij) return set_err(KFBI_ERR_ARG, "NULL argument");
    for (int k = 0; k < p->I; ++k) {
        ij[2 * k] = p->plan.irr_i[k];
        ij[2 * k + 1] = p->plan.irr_j[k];
    }
    return KFBI_OK;
}

kfbi_status kfbi_apply(kfbi_prob* p, const double* phi, double* out) {
    if (!p) return set_err(KFBI_ERR_ARG, "prob is NULL");
    if (kfbi_status s = check_ptr(phi, "phi")) return s;
    if (kfbi_status s = check_ptr(out, "out")) return s;
    HIP_TRY(hipSetDevice(p->ctx->device));
    return checked_apply(p, kOpD, phi, out);
}

kfbi_status kfbi_apply_noalloc(kfbi_prob* p, const double* phi, double* out) {
    if (!p) return set_err(KFBI_ERR_ARG, "prob is NULL");
    if (kfbi_status s = check_ptr(phi, "phi")) return s;
    if (kfbi_status s = check_ptr(out, "out")) return s;
    const int M = p->M;
    const DevPlan d = op_view(p, kOpD);
    auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
    const size_t off_s2 = 256, off_corr = off_s2 + up(sizeof(double) * M);
    const size_t off_part = off_corr + up(sizeof(double) * (size_t)d.T * 64);
    const size_t need = off_part + sizeof(double) * (size_t)p->G * M;
    if (need > kNoAllocBytes)
        return set_err(KFBI_ERR_UNSUPPORTED, "kfbi_apply_noalloc: the problem needs " + std::to_string(need) +
                                                 " bytes of scratch, more than its " + std::to_string(kNoAllocBytes));
    HIP_TRY(hipSetDevice(p->ctx->device));
    void* base = nullptr;
    if (kfbi_status e = scratch_on(p->ctx->device, &base)) return e;
    unsigned char* b = static_cast<unsigned char*>(base);
    int* flag = reinterpret_cast<int*>(b);
    double* s2 = reinterpret_cast<double*>(b + off_s2);
    double* corr_il = reinterpret_cast<double*>(b + off_corr);
    double* part = reinterpret_cast<double*>(b + off_part);
    hipStream_t s = p->ctx->stream;
    // the array keeps the last call's contents: the corrections' pad slots must
    // be zero; the flag is written by its check whatever it finds
    HIP_TRY(launch_fill((size_t)d.T * 64, 0.0, corr_il, s));
    HIP_TRY(launch_nonfinite(M, phi, flag, s));
    HIP_TRY(launch_spline(p->dp, phi, s2, flag, s));
    const JumpSrc js{phi, s2, nullptr, nullptr, nullptr, nullptr};
    HIP_TRY(launch_correct(d, js, nullptr, corr_il, nullptr, flag, s));
    HIP_TRY(launch_modes(d, corr_il, part, p->Rm, flag, s));
    HIP_TRY(launch_reduce_interp(d, js, part, p->G, out, flag, nullptr, s));
    return KFBI_OK;
}

kfbi_status kfbi_correct(kfbi_prob* p, const double* phi, const double* f_gamma, double* corr) {
    if (!p) return set_err(KFBI_ERR_ARG, "prob is NULL");
    if (kfbi_status s = check_ptr(corr, "corr")) return s;
    HIP_TRY(hipSetDevice(p->ctx->device));
    hipStream_t s = p->ctx->stream;
    JumpSrc js{phi, nullptr, f_gamma, nullptr, nullptr, nullptr};
    if (phi) {
        HIP_TRY(launch_spline(p->dp, phi, p->s2a, nullptr, s));
        js.phi_s2 = p->s2a;
    }
    if (f_gamma) {
        HIP_TRY(launch_spline(p->dp, f_gamma, p->s2b, nullptr, s));
        js.fgam_s2 = p->s2b;
    }
    HIP_TRY(launch_correct(p->dp, js, corr, nullptr, nullptr, nullptr, s));
    return KFBI_OK;
}

kfbi_status kfbi_fast_solve(kfbi_prob* p, const double* rhs, double* v) {
    if (!p) return set_err(KFBI_ERR_ARG, "prob is NULL");
    if (kfbi_status s = check_ptr(rhs, "rhs")) return s;
    if (kfbi_status s = check_ptr(v, "v")) return s;
    HIP_TRY(hipSetDevice(p->ctx->device));
    hipStream_t s = p->ctx->stream;
    HIP_TRY(launch_fill_rhs(p->dp, rhs, false, p->R, s));
    const double* V = nullptr;
    if (kfbi_status e = grid_solve(p, &V)) return e;
    HIP_TRY(launch_grid_out(p->dp, V, false, v, s));
    return KFBI_OK;
}

kfbi_status kfbi_interface_solve(kfbi_prob* p, const double* phi, const double* ftilde, const double* f_gamma,
                                 double* vgrid, double* vz) {
    if (!p) return set_err(KFBI_ERR_ARG, "prob is NULL");
    if (!vgrid && !vz) return set_err(KFBI_ERR_ARG, "no output requested");
    HIP_TRY(hipSetDevice(p->ctx->device));
    JumpSrc js{phi, nullptr, f_gamma, nullptr, nullptr, nullptr};
    return dense_interface_solve(p, false, js, ftilde, false, vgrid, false, vz);
}

kfbi_status kfbi_interface_solve_jumps(kfbi_prob* p, const double* jq, const double* jz, const double* ftilde,
                                       double* vgrid, double* vz) {
    if (!p) return set_err(KFBI_ERR_ARG, "prob is NULL");
    if (kfbi_status s = check_ptr(jq, "jq")) return s;
    if (kfbi_status s = check_ptr(jz, "jz")) return s;
    HIP_TRY(hipSetDevice(p->ctx->device));
    JumpSrc js{nullptr, nullptr, nullptr, nullptr, jq, jz};
    return dense_interface_solve(p, false, js, ftilde, false, vgrid, false, vz);
}

kfbi_status kfbi_solve(kfbi_prob* p, const double* f_grid, const double* f_gamma, const double* g, double* u_grid,
                       double* u_gamma, double* phi, int* iters, double* rel_res) {
    if (!p) return set_err(KFBI_ERR_ARG, "prob is NULL");
    for (auto [ptr, name] : {std::pair<const void*, const char*>{f_grid, "f_grid"}, {f_gamma, "f_gamma"}, {g, "g"},
                             {u_grid, "u_grid"}, {u_gamma, "u_gamma"}, {phi, "phi"}})
        if (kfbi_status s = check_ptr(ptr, name)) return s;
    HIP_TRY(hipSetDevice(p->ctx->device));
    hipStream_t s = p->ctx->stream;
    const int M = p->M;
    // g^ = g - (Y f)^+ (Sec. 2.1)
    JumpSrc jy{nullptr, nullptr, f_gamma, nullptr, nullptr, nullptr};
    if (kfbi_status e = dense_interface_solve(p, false, jy, f_grid, true, nullptr, false, p->tmpM)) return e;
    GmresBufs b = p->gm;
    HIP_TRY(launch_axpby(M, 1.0, g, -1.0, p->tmpM, b.ghat, s));
    // GMRES (Alg. 5): every step is one K_D apply plus one orthogonalisation
    GmresState st{};
    if (kfbi_status e = run_gmres(p, kOpD, nullptr, phi, p->tol, p->max_iter, &st)) return e;
    if (st.converged == kGmNonfinite) return set_err(KFBI_ERR_NONFINITE, "NaN or Inf in f, f_gamma, g or phi");
    // u = W phi + Y f
    JumpSrc jf{b.phi, nullptr, f_gamma, nullptr, nullptr, nullptr};
    if (kfbi_status e = dense_interface_solve(p, false, jf, f_grid, true, u_grid, true, u_gamma)) return e;
    HIP_TRY(hipMemcpyAsync(phi, b.phi, M * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (iters) *iters = st.it;
    if (rel_res) *rel_res = st.relres;
    if (st.converged == 1) return KFBI_OK;
    return set_err(KFBI_NOT_CONVERGED, "GMRES reached the iteration cap");
}

kfbi_status kfbi_gmres(kfbi_prob* p, const double* rhs, double* phi, double tol, int max_iter, int* iters,
                       int* applies, double* rel_res) {
    return gmres_call(p, kOpD, rhs, phi, tol, max_iter, iters, applies, rel_res);
}

kfbi_status kfbi_richardson(kfbi_prob* p, const double* rhs, double* phi, double gamma, double tol, int max_iter,
                           int* iters, double* rel_res) {
    if (!(gamma > 0.0)) return set_err(KFBI_ERR_ARG, "gamma must be positive");
    IterState st{};
    if (kfbi_status e = run_iters(p, kRich, rhs, phi, gamma, tol, max_iter, &st)) return e;
    if (iters) *iters = st.it;
    if (rel_res) *rel_res = st.relres;
    if (st.done == 1) return KFBI_OK;
    return set_err(KFBI_NOT_CONVERGED, "Richardson reached the iteration cap");
}

kfbi_status kfbi_bicgstab(kfbi_prob* p, const double* rhs, double* phi, double tol, int max_iter, int* iters,
                          int* applies, double* rel_res) {
    IterState st{};
    if (kfbi_status e = run_iters(p, kBicg, rhs, phi, 0.0, tol, max_iter, &st)) return e;
    if (iters) *iters = st.it;
    // the initial residual, two per iteration (one in a half-way stop), the final true residual
    if (applies) *applies = 2 + 2 * st.it - st.half;
    if (rel_res) *rel_res = st.relres;
    if (st.done == 1) return KFBI_OK;
    return set_err(KFBI_NOT_CONVERGED, "BiCGSTAB reached the iteration cap");
}

kfbi_status kfbi_solve_method(kfbi_prob* p, int method, double relax, const double* f_grid, const double* f_gamma,
                              const double* g, double* u_grid, double* u_gamma, double* phi, int* iters,
                              double* rel_res) {
    if (!p) return set_err(KFBI_ERR_ARG, "prob is NULL");
    if (method == KFBI_GMRES) return kfbi_solve(p, f_grid, f_gamma, g, u_grid, u_gamma, phi, iters, rel_res);
    if (method != KFBI_BICGSTAB && method != KFBI_RICHARDSON) return set_err(KFBI_ERR_ARG, "unknown method");
    if (method == KFBI_RICHARDSON && !(relax > 0.0)) return set_err(KFBI_ERR_ARG, "relax must be positive");
    for (auto [ptr, name] : {std::pair<const void*, const char*>{f_grid, "f_grid"}, {f_gamma, "f_gamma"}, {g, "g"},
                             {u_grid, "u_grid"}, {u_gamma, "u_gamma"}, {phi, "phi"}})
        if (kfbi_status s = check_ptr(ptr, name)) return s;
    HIP_TRY(hipSetDevice(p->ctx->device));
    hipStream_t s = p->ctx->stream;
    const int M = p->M;
    JumpSrc jy{nullptr, nullptr, f_gamma, nullptr, nullptr, nullptr};
    if (kfbi_status e = dense_interface_solve(p, false, jy, f_grid, true, nullptr, false, p->tmpM)) return e;
    HIP_TRY(launch_axpby(M, 1.0, g, -1.0, p->tmpM, p->tmpM, s));
    IterState st{};
    if (kfbi_status e = run_iters(p, method == KFBI_BICGSTAB ? kBicg : kRich, p->tmpM, phi, relax, p->tol,
                                  p->max_iter, &st))
        return e;
    JumpSrc jf{phi, nullptr, f_gamma, nullptr, nullptr, nullptr};
    if (kfbi_status e = dense_interface_solve(p, false, jf, f_grid, true, u_grid, true, u_gamma)) return e;
    HIP_TRY(hipStreamSynchronize(s));
    if (iters) *iters = st.it;
    if (rel_res) *rel_res = st.relres;
    if (st.done == 1) return KFBI_OK;
    return set_err(KFBI_NOT_CONVERGED, "the iteration reached its cap");
}

kfbi_status kfbi_apply_neumann(kfbi_prob* p, const double* psi, double* out) {
    if (!p) return set_err(KFBI_ERR_ARG, "prob is NULL");
    if (kfbi_status s = check_ptr(psi, "psi")) return s;
    if (kfbi_status s = check_ptr(out, "out")) return s;
    HIP_TRY(hipSetDevice(p->ctx->device));
    return checked_apply(p, kOpN, psi, out);
}

kfbi_status kfbi_interface_solve_neumann(kfbi_prob* p, const double* psi, const double* ftilde, const double* f_gamma,
                                         double* vgrid, double* vz, double* dnz) {
    if (!p) return set_err(KFBI_ERR_ARG, "prob is NULL");
    if (!vgrid && !vz && !dnz) return set_err(KFBI_ERR_ARG, "no output requested");
    HIP_TRY(hipSetDevice(p->ctx->device));
    JumpSrc js{psi, nullptr, f_gamma, nullptr, nullptr, nullptr};
    return dense_interface_solve(p, true, js, ftilde, false, vgrid, false, vz, dnz);
}

kfbi_status kfbi_gmres_neumann(kfbi_prob* p, const double* rhs, double* psi, double tol, int max_iter, int* iters,
                               int* applies, double* rel_res) {
    return gmres_call(p, kOpN, rhs, psi, tol, max_iter, iters, applies, rel_res);
}

kfbi_status kfbi_solve_neumann(kfbi_prob* p, const double* f_grid, const double* f_gamma, const double* g_n,
                               double* u_grid, double* u_gamma, double* dn_gamma, double* psi, int* iters,
                               double* rel_res) {
    const NeumannIO io{f_grid, f_gamma, g_n, u_grid, u_gamma, dn_gamma, psi};
    if (kfbi_status e = neumann_check(p, io)) return e;
    HIP_TRY(hipSetDevice(p->ctx->device));
    if (kfbi_status e = neumann_prepare(p, io)) return e;
    // GMRES on K_N psi = g^: every step is one K_N apply plus one orthogonalisation
    GmresState st{};
    if (kfbi_status e = run_gmres(p, kOpN, nullptr, psi, p->tol, p->max_iter, &st)) return e;
    if (st.converged == kGmNonfinite) return set_err(KFBI_ERR_NONFINITE, "NaN or Inf in f, f_gamma, g_n or psi");
    if (kfbi_status e = neumann_finish(p, io)) return e;
    HIP_TRY(hipStreamSynchronize(p->ctx->stream));
    if (iters) *iters = st.it;
    if (rel_res) *rel_res = st.relres;
    if (st.converged == 1) return KFBI_OK;
    return set_err(KFBI_NOT_CONVERGED, "GMRES reached the iteration cap");
}

kfbi_status kfbi_prob_set_reorth(kfbi_prob* p, double eta) {
    if (!p) return set_err(KFBI_ERR_ARG, "prob is NULL");
    if (!(eta >= 0.0 && eta <= 1.0)) return set_err(KFBI_ERR_ARG, "eta must lie in [0, 1]");
    p->reorth = eta;
    return KFBI_OK;
}

kfbi_status kfbi_set_timing(kfbi_prob* p, int on) {
    if (!p) return set_err(KFBI_ERR_ARG, "prob is NULL");
    p->timing = on != 0;
    if (p->timing) p->t_count = 0;
    return KFBI_OK;
}

kfbi_status kfbi_apply_timing(kfbi_prob* p, double* a, double* b, double* c, int* count) {
    if (!p) return set_err(KFBI_ERR_ARG, "prob is NULL");
    HIP_TRY(hipStreamSynchronize(p->ctx->stream));
    double acc[3] = {0, 0, 0};
    for (int k = 0; k < p->t_count; ++k) {
        for (int q = 0; q < 3; ++q) {
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, p->ev[6 * k + 2 * q], p->ev[6 * k + 2 * q + 1]));
            acc[q] += 1e3 * ms;
        }
    }
    const double k = p->t_count ? 1.0 / p->t_count : 0.0;
    if (a) *a = acc[0] * k;
    if (b) *b = acc[1] * k;
    if (c) *c = acc[2] * k;
    if (count) *count = p->t_count;
    return KFBI_OK;
}

// ---------------------------------------------------------------- tile shapes

}  // extern "C"

namespace {

bool tiles_valid(const kfbi_prob* p, int Rm, int B) {
    if (Rm < 1 || Rm > kMaxModesPerGroup || (Rm & (Rm - 1))) return false;
    if (modes_lds_bytes(p->N, Rm) > p->ctx->lds_max) return false;
    if ((p->n + Rm - 1) / Rm > p->Gcap) return false;
    return dst_tile_ok(p->N, B, cpx_bytes(p->precision), p->ctx->lds_max);
}

void drop_graph(kfbi_prob* p) {
    for (int op = 0; op < 2; ++op)
        for (int k = 0; k < kfbi_prob::kGraphSizes; ++k) {
            if (p->gexec[op][k]) hipGraphExecDestroy(p->gexec[op][k]);
            p->gexec[op][k] = nullptr;
            p->graph_failed[op][k] = false;
        }
}

// mean time in microseconds of `reps` runs of `body` (after one warm-up run)
template <class F>
kfbi_status time_us(hipStream_t s, int reps, double* us, F body) {
    if (kfbi_status e = body()) return e;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        hipEventDestroy(e0);
        return set_err(KFBI_ERR_DEVICE, "event creation failed");
    }
    kfbi_status st = KFBI_OK;
    float ms = 0.f;
    if (hipEventRecord(e0, s) != hipSuccess) st = set_err(KFBI_ERR_DEVICE, "event record failed");
    for (int k = 0; k < reps && st == KFBI_OK; ++k) st = body();
    if (st == KFBI_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                          hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        st = set_err(KFBI_ERR_DEVICE, "event timing failed");
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    *us = 1e3 * ms / reps;
    return st;
}

}  // namespace

extern "C" {

kfbi_status kfbi_prob_get_tiles(const kfbi_prob* p, kfbi_tiles* out) {
    if (!p || !out) return set_err(KFBI_ERR_ARG, "NULL argument");
    out->modes_per_group = p->Rm;
    out->modes_groups = p->G;
    out->dst_cols = p->dstB;
    out->apply_us = p->tuned_apply_us;
    out->grid_solve_us = p->tuned_grid_us;
    return KFBI_OK;
}

kfbi_status kfbi_prob_set_tiles(kfbi_prob* p, const kfbi_tiles* t) {
    if (!p || !t) return set_err(KFBI_ERR_ARG, "NULL argument");
    if (!tiles_valid(p, t->modes_per_group, t->dst_cols))
        return set_err(KFBI_ERR_ARG, "tile shape not valid for this problem");
    HIP_TRY(hipSetDevice(p->ctx->device));
    HIP_TRY(hipStreamSynchronize(p->ctx->stream));      // a replayed graph may still use the old shape
    p->Rm = t->modes_per_group;
    p->G = (p->n + p->Rm - 1) / p->Rm;
    p->dstB = t->dst_cols;
    drop_graph(p);
    return KFBI_OK;
}

kfbi_status kfbi_prob_autotune(kfbi_prob* p, int reps, kfbi_tiles* out) {
    if (!p || !out) return set_err(KFBI_ERR_ARG, "NULL argument");
    if (reps <= 0) reps = 10;
    HIP_TRY(hipSetDevice(p->ctx->device));
    hipStream_t s = p->ctx->stream;
    HIP_TRY(hipStreamSynchronize(s));
    drop_graph(p);
    // a zero density in tmpM with its spline in s2a: the values do not change the work
    HIP_TRY(hipMemsetAsync(p->tmpM, 0, sizeof(double) * p->M, s));
    HIP_TRY(hipMemsetAsync(p->s2a, 0, sizeof(double) * p->M, s));
    double best = 1e300;
    const int r0 = p->Rm;
    int br = r0;
    for (int Rm : {r0 / 2, r0, 2 * r0}) {
        if (!tiles_valid(p, Rm, p->dstB)) continue;
        p->Rm = Rm;
        p->G = (p->n + Rm - 1) / Rm;
        double us = 0;
        if (kfbi_status e = time_us(s, reps, &us,
                                    [&] { return sparse_apply(p, kOpD, p->tmpM, p->s2a, p->s2b, nullptr, nullptr, s); })) {
            p->Rm = r0;
            p->G = (p->n + r0 - 1) / r0;
            return e;
        }
        if (us < best) {
            best = us;
            br = Rm;
        }
    }
    p->Rm = br;
    p->G = (p->n + br - 1) / br;
    p->tuned_apply_us = best;
    double bestg = 1e300;
    int bb = p->dstB;
    const double* V = nullptr;
    for (int B : {4, 8, 16}) {
        if (!tiles_valid(p, p->Rm, B)) continue;
        p->dstB = B;
        double us = 0;
        if (kfbi_status e = time_us(s, reps, &us, [&] {
                HIP_TRY(launch_fill_rhs(p->dp, nullptr, false, p->R, s));
                return grid_solve(p, &V);
            })) {
            p->dstB = bb;
            return e;
        }
        if (us < bestg) {
            bestg = us;
            bb = B;
        }
    }
    p->dstB = bb;
    p->tuned_grid_us = bestg;
    return kfbi_prob_get_tiles(p, out);
}

// ---------------------------------------------------------------- batches

}  // extern "C"

struct kfbi_batch {
    kfbi_ctx* ctx = nullptr;
    int max_slots = 0, mmax = 0;
    size_t budget = 0, used = 0;
    std::vector<kfbi_prob*> slot;
    std::vector<size_t> slot_bytes;
    std::vector<SlotDev> h_slots;
    SlotDev* d_slots = nullptr;
    int* d_counts = nullptr;
    int2* d_corr = nullptr;
    int2* d_mode = nullptr;
    int2* d_cp = nullptr;
    int2* d_gm = nullptr;
    int* d_live = nullptr;
    int cap_corr = 0, cap_mode = 0, cap_cp = 0, cap_gm = 0;
    std::vector<int2> h_corr, h_mode, h_cp, h_gm;
    std::vector<int> h_live;
    int h_counts[kBatchCounts] = {0, 0, 0, 0, 0};
    // pinned staging of the uploads, reused once the event says the stream has
    // consumed the previous upload
    char* stage = nullptr;
    size_t stage_cap = 0;
    hipEvent_t up_ev = nullptr;
    hipGraphExec_t gexec = nullptr;
    bool graph_failed = false;
    static constexpr int kGraphSteps = 8;
};

namespace {

void batch_free_lists(kfbi_batch* B) {
    for (void* q : {(void*)B->d_corr, (void*)B->d_mode, (void*)B->d_cp, (void*)B->d_gm})
        if (q) hipFree(q);
    B->d_corr = nullptr;
    B->d_mode = nullptr;
    B->d_cp = nullptr;
    B->d_gm = nullptr;
    B->cap_corr = B->cap_mode = B->cap_cp = B->cap_gm = 0;
}

kfbi_status batch_grow(hipStream_t s, int2** d, int* cap, size_t need) {
    if ((size_t)*cap >= need) return KFBI_OK;
    size_t nc = std::max<size_t>(need, 2 * (size_t)*cap);
    if (*d) {
        HIP_TRY(hipStreamSynchronize(s));   // queued launches may still read the old list
        hipFree(*d);
    }
    *d = nullptr;
    if (hipMalloc((void**)d, nc * sizeof(int2)) != hipSuccess) {
        hipGetLastError();
        *cap = 0;
        return set_err(KFBI_ERR_OOM, "batch work list allocation failed");
    }
    *cap = (int)nc;
    return KFBI_OK;
}

// Rebuild the work lists of the live slots and upload them (stream ordered).
kfbi_status batch_rebuild(kfbi_batch* B) {
    B->h_corr.clear();
    B->h_mode.clear();
    B->h_cp.clear();
    B->h_gm.clear();
    B->h_live.clear();
    for (int s = 0; s < B->max_slots; ++s) {
        kfbi_prob* p = B->slot[s];
        if (!p) continue;
        B->h_live.push_back(s);
        for (int r = 0; r < p->I; r += 256) B->h_corr.push_back(make_int2(s, r));
        for (int b = 0; b < p->Gs; ++b) B->h_mode.push_back(make_int2(s, b));
        for (int c = 0; c < p->M; c += 64) B->h_cp.push_back(make_int2(s, c));
        for (int c = 0; c < p->gm.gc; ++c) B->h_gm.push_back(make_int2(s, c));
    }
    const int2* old[4] = {B->d_corr, B->d_mode, B->d_cp, B->d_gm};
    hipStream_t gs = B->ctx->stream;
    if (kfbi_status e = batch_grow(gs, &B->d_corr, &B->cap_corr, std::max<size_t>(B->h_corr.size(), 1))) return e;
    if (kfbi_status e = batch_grow(gs, &B->d_mode, &B->cap_mode, std::max<size_t>(B->h_mode.size(), 1))) return e;
    if (kfbi_status e = batch_grow(gs, &B->d_cp, &B->cap_cp, std::max<size_t>(B->h_cp.size(), 1))) return e;
    if (kfbi_status e = batch_grow(gs, &B->d_gm, &B->cap_gm, std::max<size_t>(B->h_gm.size(), 1))) return e;
    if (old[0] != B->d_corr || old[1] != B->d_mode || old[2] != B->d_cp || old[3] != B->d_gm) {
        // the captured graph holds the old list addresses
        if (B->gexec) hipGraphExecDestroy(B->gexec);
        B->gexec = nullptr;
    }
    hipStream_t s = B->ctx->stream;
    B->h_counts[0] = (int)B->h_corr.size();
    B->h_counts[1] = (int)B->h_mode.size();
    B->h_counts[2] = (int)B->h_cp.size();
    B->h_counts[3] = (int)B->h_live.size();
    B->h_counts[4] = (int)B->h_gm.size();
    const size_t nb = sizeof(int2) * (B->h_corr.size() + B->h_mode.size() + B->h_cp.size() + B->h_gm.size()) +
                      sizeof(int) * (B->h_live.size() + kBatchCounts) + sizeof(SlotDev) * B->max_slots;
    HIP_TRY(hipEventSynchronize(B->up_ev));
    if (nb > B->stage_cap) {
        if (B->stage) hipHostFree(B->stage);
        B->stage = nullptr;
        B->stage_cap = 0;
        HIP_TRY(hipHostMalloc((void**)&B->stage, 2 * nb));
        B->stage_cap = 2 * nb;
    }
    // upload, ordered on the stream after the work that used the previous lists
    char* q = B->stage;
    auto put = [&](void* dst, const void* src, size_t bytes) -> kfbi_status {
        if (!bytes) return KFBI_OK;
        std::memcpy(q, src, bytes);
        HIP_TRY(hipMemcpyAsync(dst, q, bytes, hipMemcpyHostToDevice, s));
        q += bytes;
        return KFBI_OK;
    };
    kfbi_status e = KFBI_OK;
    if ((e = put(B->d_corr, B->h_corr.data(), B->h_corr.size() * sizeof(int2))) ||
        (e = put(B->d_mode, B->h_mode.data(), B->h_mode.size() * sizeof(int2))) ||
        (e = put(B->d_cp, B->h_cp.data(), B->h_cp.size() * sizeof(int2))) ||
        (e = put(B->d_gm, B->h_gm.data(), B->h_gm.size() * sizeof(int2))) ||
        (e = put(B->d_live, B->h_live.data(), B->h_live.size() * sizeof(int))) ||
        (e = put(B->d_counts, B->h_counts, sizeof B->h_counts)) ||
        (e = put(B->d_slots, B->h_slots.data(), sizeof(SlotDev) * B->max_slots)))
        return e;
    HIP_TRY(hipEventRecord(B->up_ev, s));
    return KFBI_OK;
}

BatchWork batch_work(const kfbi_batch* B) {
    BatchWork w;
    w.counts = B->d_counts;
    w.corr_items = B->d_corr;
    w.mode_items = B->d_mode;
    w.cp_items = B->d_cp;
    w.live = B->d_live;
    w.gm_items = B->d_gm;
    w.max_live = B->max_slots;
    return w;
}

kfbi_status batch_enqueue_steps(kfbi_batch* B, int nsteps, hipStream_t s) {
    for (int k = 0; k < nsteps; ++k)
        HIP_TRY(launch_batch_step(B->d_slots, batch_work(B), B->ctx->num_cu, s));
    return KFBI_OK;
}

void batch_ensure_graph(kfbi_batch* B) {
    if (B->gexec || B->graph_failed) return;
    B->graph_failed = !record_graph(B->ctx->stream, &B->gexec, [&](hipStream_t s) {
        return batch_enqueue_steps(B, kfbi_batch::kGraphSteps, s);
    });
}

size_t batch_extra_bytes(int n, int m) {
    const int r = batch_modes_per_group(n);
    const int Gs = (n - 1 + r - 1) / r;
    return sizeof(double) * (size_t)m * Gs;
}

}  // namespace

extern "C" {

kfbi_status kfbi_batch_estimate_bytes(int n, int m, int restart, size_t* bytes) {
    if (!bytes || n < 64 || m < 3) return set_err(KFBI_ERR_ARG, "bad arguments");
    if (restart <= 0) restart = 50;
    restart = std::min(restart, kMaxRestart);
    // plan: crossings and irregular nodes are O(perimeter / h); bound them by 8 n
    const size_t nq = 8 * (size_t)n, ni = 8 * (size_t)n;
    const size_t slots = ni + 64 * (size_t)(kSlots + 64);                  // interleaved table, padded
    size_t b = nq * (sizeof(PointGeom) + 4) + (size_t)m * 256 + ni * 80 + slots * 12 +
               (size_t)(n + 1) * (n + 1) + (size_t)n * (sizeof(ModeConst) + 16) + 4096;
    b += 2 * sizeof(double) * (size_t)n * n;                                  // dense-path grids
    b += sizeof(double) * ((size_t)(restart + 1) * (m + restart) + 16 * (size_t)m +
                           gm_part_size(restart, gm_chunks(m), gm_chunks64(m)) + restart + 2);   // GMRES
    b += sizeof(double) * (size_t)m * 512;                                    // single-path partials
    b += batch_extra_bytes(n, m);
    *bytes = b;
    return KFBI_OK;
}

kfbi_status kfbi_batch_create(kfbi_ctx* ctx, int max_slots, int m_max, size_t budget, kfbi_batch** out) {
    if (!ctx || !out || max_slots < 1 || max_slots > 1024 || m_max < 3 || m_max > kMaxSamples)
        return set_err(KFBI_ERR_ARG, "bad batch arguments");
    HIP_TRY(hipSetDevice(ctx->device));
    if (modes_b_lds_bytes() > ctx->lds_max)
        return set_err(KFBI_ERR_UNSUPPORTED, "the batched fast solve does not fit this device's LDS");
    kfbi_batch* B = new (std::nothrow) kfbi_batch;
    if (!B) return set_err(KFBI_ERR_ARG, "host allocation failed");
    B->ctx = ctx;
    B->max_slots = max_slots;
    B->mmax = m_max;
    B->budget = budget;
    B->slot.assign(max_slots, nullptr);
    B->slot_bytes.assign(max_slots, 0);
    B->h_slots.resize(max_slots);
    bool ok = hipEventCreateWithFlags(&B->up_ev, hipEventDisableTiming) == hipSuccess &&
              hipMalloc((void**)&B->d_slots, sizeof(SlotDev) * max_slots) == hipSuccess &&
              hipMalloc((void**)&B->d_counts, sizeof(int) * kBatchCounts) == hipSuccess &&
              hipMalloc((void**)&B->d_live, sizeof(int) * max_slots) == hipSuccess;
    if (!ok) {
        hipGetLastError();
        kfbi_batch_destroy(B);
        return set_err(KFBI_ERR_OOM, "batch allocation failed");
    }
    if (kfbi_status e = batch_rebuild(B)) {
        kfbi_batch_destroy(B);
        return e;
    }
    *out = B;
    return KFBI_OK;
}

kfbi_status kfbi_batch_destroy(kfbi_batch* B) {
    if (!B) return KFBI_OK;
    hipSetDevice(B->ctx->device);
    hipStreamSynchronize(B->ctx->stream);
    if (B->gexec) hipGraphExecDestroy(B->gexec);
    batch_free_lists(B);
    for (void* q : {(void*)B->d_slots, (void*)B->d_counts, (void*)B->d_live})
        if (q) hipFree(q);
    if (B->stage) hipHostFree(B->stage);
    if (B->up_ev) hipEventDestroy(B->up_ev);
    delete B;
    return KFBI_OK;
}

kfbi_status kfbi_batch_admit(kfbi_batch* B, kfbi_prob* p, const double* f_grid, const double* f_gamma,
                             const double* g, int* slot) {
    if (!B || !p || !slot) return set_err(KFBI_ERR_ARG, "NULL argument");
    for (auto [ptr, name] : {std::pair<const void*, const char*>{f_grid, "f_grid"}, {f_gamma, "f_gamma"}, {g, "g"}})
        if (kfbi_status s = check_ptr(ptr, name)) return s;
    if (p->ctx != B->ctx) return set_err(KFBI_ERR_ARG, "problem and batch use different contexts");
    if (p->N > kBatchNmax || p->M > B->mmax)
        return set_err(KFBI_ERR_UNSUPPORTED, "problem exceeds the batch's grid or sample limit");
    for (int s = 0; s < B->max_slots; ++s)
        if (B->slot[s] == p) return set_err(KFBI_ERR_ARG, "problem already admitted");
    int free_slot = -1;
    for (int s = 0; s < B->max_slots && free_slot < 0; ++s)
        if (!B->slot[s]) free_slot = s;
    const size_t need = p->bytes + (p->partial_b ? 0 : batch_extra_bytes(p->N, p->M));
    if (B->budget && need > B->budget) return set_err(KFBI_ERR_UNSUPPORTED, "problem larger than the batch budget");
    if (free_slot < 0) return set_err(KFBI_ERR_BUDGET, "no free slot");
    if (B->budget && B->used + need > B->budget) return set_err(KFBI_ERR_BUDGET, "over the memory budget for now");
    HIP_TRY(hipSetDevice(B->ctx->device));
    hipStream_t s = B->ctx->stream;
    if (!p->partial_b) {
        const int r = batch_modes_per_group(p->N);
        p->Gs = (p->n + r - 1) / r;
        if (kfbi_status e = dev_alloc(p, &p->partial_b, (size_t)p->M * p->Gs)) return e;
    }
    // g^ = g - (Y f)^+ and a fresh GMRES state (phi_0 = 0)
    JumpSrc jy{nullptr, nullptr, f_gamma, nullptr, nullptr, nullptr};
    if (kfbi_status e = dense_interface_solve(p, false, jy, f_grid, true, nullptr, false, p->tmpM)) return e;
    GmresBufs b = p->gm;
    HIP_TRY(launch_axpby(p->M, 1.0, g, -1.0, p->tmpM, b.ghat, s));
    // the state and the first Arnoldi input (phi_0 = 0: the residual is g^);
    // the batch's own correction stage makes its corrections
    HIP_TRY(launch_gmres_start(nullptr, p->dp.taps, p->M, b, nullptr, nullptr, p->tol, p->max_iter, p->reorth,
                               nullptr, nullptr, s));
    p->st_host = GmresState{};
    SlotDev& S = B->h_slots[free_slot];
    S.p = p->dp;
    S.b = b;
    S.corr_il = p->corr_il;
    S.partial = p->partial_b;
    S.Gs = p->Gs;
    S.pad = 0;
    p->b_fgrid = f_grid;
    p->b_fgam = f_gamma;
    B->slot[free_slot] = p;
    B->slot_bytes[free_slot] = p->bytes;
    B->used += p->bytes;
    if (kfbi_status e = batch_rebuild(B)) return e;
    *slot = free_slot;
    return KFBI_OK;
}

kfbi_status kfbi_batch_step(kfbi_batch* B, int nsteps) {
    if (!B || nsteps < 0) return set_err(KFBI_ERR_ARG, "bad arguments");
    if (B->h_live.empty() || nsteps == 0) return KFBI_OK;
    HIP_TRY(hipSetDevice(B->ctx->device));
    batch_ensure_graph(B);
    const int K = kfbi_batch::kGraphSteps;
    for (int done = 0; done < nsteps; done += K) {
        if (B->gexec && nsteps - done >= K) {
            HIP_TRY(hipGraphLaunch(B->gexec, B->ctx->stream));
        } else if (kfbi_status e = batch_enqueue_steps(B, std::min(K, nsteps - done), B->ctx->stream)) {
            return e;
        }
    }
    return KFBI_OK;
}

kfbi_status kfbi_batch_poll(kfbi_batch* B, int* state, int* iters, double* rel_res) {
    if (!B) return set_err(KFBI_ERR_ARG, "batch is NULL");
    HIP_TRY(hipSetDevice(B->ctx->device));
    hipStream_t s = B->ctx->stream;
    for (int k = 0; k < B->max_slots; ++k)
        if (B->slot[k]) HIP_TRY(hipMemcpyAsync(&B->slot[k]->st_host, B->slot[k]->gm.st, sizeof(GmresState),
                                               hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int k = 0; k < B->max_slots; ++k) {
        const kfbi_prob* p = B->slot[k];
        if (state) state[k] = !p ? -2 : p->st_host.converged == kGmNonfinite ? -3 : p->st_host.converged;
        if (iters) iters[k] = p ? p->st_host.it : 0;
        if (rel_res) rel_res[k] = p ? p->st_host.relres : 0.0;
    }
    return KFBI_OK;
}

kfbi_status kfbi_batch_finish(kfbi_batch* B, int slot, double* u_grid, double* u_gamma, double* phi) {
    if (!B || slot < 0 || slot >= B->max_slots || !B->slot[slot]) return set_err(KFBI_ERR_ARG, "no such slot");
    for (auto [ptr, name] : {std::pair<const void*, const char*>{u_grid, "u_grid"}, {u_gamma, "u_gamma"}, {phi, "phi"}})
        if (kfbi_status e = check_ptr(ptr, name)) return e;
    HIP_TRY(hipSetDevice(B->ctx->device));
    kfbi_prob* p = B->slot[slot];
    hipStream_t s = B->ctx->stream;
    // a slot that stopped on a NaN or Inf (as the last poll saw it) is released
    // with nothing written
    const bool bad = p->st_host.converged == kGmNonfinite;
    if (!bad) {
        JumpSrc jf{p->gm.phi, nullptr, p->b_fgam, nullptr, nullptr, nullptr};
        if (kfbi_status e = dense_interface_solve(p, false, jf, p->b_fgrid, true, u_grid, true, u_gamma)) return e;
        HIP_TRY(hipMemcpyAsync(phi, p->gm.phi, p->M * sizeof(double), hipMemcpyDeviceToDevice, s));
    }
    B->used -= B->slot_bytes[slot];
    B->slot[slot] = nullptr;
    B->slot_bytes[slot] = 0;
    p->b_fgrid = p->b_fgam = nullptr;
    if (kfbi_status e = batch_rebuild(B)) return e;
    return bad ? set_err(KFBI_ERR_NONFINITE, "NaN or Inf in the slot's f, f_gamma or g") : KFBI_OK;
}

kfbi_status kfbi_batch_info(const kfbi_batch* B, int* live, size_t* bytes) {
    if (!B) return set_err(KFBI_ERR_ARG, "batch is NULL");
    if (live) *live = (int)B->h_live.size();
    if (bytes) *bytes = B->used;
    return KFBI_OK;
}

}  // extern "C"
