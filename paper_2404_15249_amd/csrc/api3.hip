// C ABI of the three-dimensional problem (include/kfbi.h, kfbi3_*): the
// ellipsoid Dirichlet problem on the 7-point grid, its K_D apply, interface
// solves and the device-resident GMRES solve.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <string>
#include <vector>

#include "api_common.h"
#include "gmres.h"
#include "k3.h"
#include "plan3.h"

using namespace kfbi;

struct kfbi_prob3 {
    kfbi_ctx* ctx = nullptr;
    Plan3Host plan;
    double kappa = 0, tol = 1e-10;
    int restart = 50, max_iter = 500;
    int N = 0, M = 0, I = 0;
    DevPlan3 dp{};
    std::vector<void*> allocs;
    size_t bytes = 0;
    double* G = nullptr;        // N^3 grid, interior layout
    double* J = nullptr;        // 10 M jumps
    double* tmpM = nullptr;     // M
    double* zeroM = nullptr;    // M zeros (the density of Y f)
    int* d_flag = nullptr;      // 1: the density checked by kfbi3_apply holds a NaN or Inf
    int h_flag = 0;
    int dstB = 16;
    GmresBufs gm{};
    GmresState st_host{};
    static constexpr int kGraphSteps = 8;
    hipGraphExec_t gexec = nullptr;
    bool graph_failed = false;
};

namespace {

template <class T>
kfbi_status alloc3(kfbi_prob3* p, T** out, size_t count) {
    void* d = nullptr;
    const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
    if (hipMalloc(&d, bytes) != hipSuccess) {
        hipGetLastError();
        return set_err(KFBI_ERR_OOM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    }
    p->allocs.push_back(d);
    p->bytes += bytes;
    *out = static_cast<T*>(d);
    return KFBI_OK;
}

template <class T>
kfbi_status upload3(kfbi_prob3* p, const T** out, const std::vector<T>& v) {
    T* d = nullptr;
    if (kfbi_status s = alloc3(p, &d, v.size())) return s;
    if (!v.empty() && hipMemcpy(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
        return set_err(KFBI_ERR_DEVICE, "upload failed");
    *out = d;
    return KFBI_OK;
}

void free3(kfbi_prob3* p) {
    if (p->gexec) hipGraphExecDestroy(p->gexec);
    for (void* a : p->allocs) hipFree(a);
    delete p;
}

// one interface solve: jumps from (phi, fgam), the masked base right-hand side
// f (null: zero), correction, fast solve; v+ at the control points into vz
// (null: skipped), the grid solution into vgrid (null: skipped)
kfbi_status interface3(kfbi_prob3* p, const double* phi, const double* f, const double* fgam, double* vgrid,
                       bool mask, double* vz) {
    hipStream_t s = p->ctx->stream;
    HIP_TRY(launch_jumps3(p->dp, phi ? phi : p->zeroM, fgam, p->J, nullptr, s));
    HIP_TRY(launch_fill3(p->dp, f, p->G, nullptr, s));
    HIP_TRY(launch_correct3(p->dp, p->J, p->G, nullptr, s));
    HIP_TRY(launch_solve3(p->dp, p->G, p->dstB, nullptr, s));
    if (vz) HIP_TRY(launch_interp3(p->dp, p->G, p->J, vz, nullptr, s));
    if (vgrid) HIP_TRY(launch_grid_out3(p->dp, p->G, mask, vgrid, s));
    return KFBI_OK;
}

kfbi_status enqueue_steps3(kfbi_prob3* p, int nsteps, hipStream_t s) {
    GmresBufs b = p->gm;
    const int* skip = &b.st->converged;
    for (int k = 0; k < nsteps; ++k) {
        HIP_TRY(launch_jumps3(p->dp, b.xcur, nullptr, p->J, skip, s));
        HIP_TRY(launch_fill3(p->dp, nullptr, p->G, skip, s));
        HIP_TRY(launch_correct3(p->dp, p->J, p->G, skip, s));
        HIP_TRY(launch_solve3(p->dp, p->G, p->dstB, skip, s));
        HIP_TRY(launch_interp3(p->dp, p->G, p->J, nullptr, &b, s));
        HIP_TRY(launch_gmres_step(nullptr, p->M, b, s));
    }
    return KFBI_OK;
}

// Restarted GMRES on K_D phi = ghat (ghat already in gm.ghat), as for the
// curve problem: batches of steps replayed from one recorded graph, the
// host polling the device state between batches when tol > 0.
kfbi_status run_gmres3(kfbi_prob3* p, const double* phi_in, double tol, int max_iter, GmresState* out) {
    hipStream_t s = p->ctx->stream;
    GmresBufs b = p->gm;
    // the state and the first K_D input on the device (gm_start)
    HIP_TRY(launch_gmres_start(nullptr, nullptr, p->M, b, nullptr, phi_in, tol, max_iter, kGmReorthDefault, nullptr,
                               nullptr, s));
    if (!p->gexec && !p->graph_failed)
        p->graph_failed = !record_graph(s, &p->gexec,
                                        [&](hipStream_t st) { return enqueue_steps3(p, kfbi_prob3::kGraphSteps, st); });
    // Arnoldi steps and one residual step per cycle end; a nonzero guess takes
    // one residual step more, found in the last poll
    const int m = std::max(1, p->restart);
    int max_steps = max_iter + (max_iter + m - 1) / m;
    bool extended = false;
    const int B = kfbi_prob3::kGraphSteps;
    GmresState& st = p->st_host;
    for (int done = 0;;) {
        if (done >= max_steps) {
            if (st.converged || extended) break;
            extended = true;
            max_steps += 1;
        }
        const int n = std::min(B, max_steps - done);
        if (p->gexec && n == B) {
            HIP_TRY(hipGraphLaunch(p->gexec, s));
        } else if (kfbi_status e = enqueue_steps3(p, n, s)) {
            return e;
        }
        done += n;
        if (tol > 0 || done >= max_steps) {
            HIP_TRY(hipMemcpyAsync(&st, b.st, sizeof st, hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            if (st.converged) break;
        }
    }
    *out = st;
    return KFBI_OK;
}

}  // namespace

extern "C" {

kfbi_status kfbi3_prob_create(kfbi_ctx* ctx, const kfbi_desc3* d, kfbi_prob3** out) {
    if (!ctx || !d || !out) return set_err(KFBI_ERR_ARG, "NULL argument");
    *out = nullptr;
    if (!(d->hi > d->lo)) return set_err(KFBI_ERR_ARG, "empty box");
    if (!(d->kappa >= 0.0)) return set_err(KFBI_ERR_ARG, "kappa must be >= 0");
    const int restart = d->restart > 0 ? d->restart : 50;
    if (restart > kMaxRestart) return set_err(KFBI_ERR_ARG, "restart exceeds " + std::to_string(kMaxRestart));
    HIP_TRY(hipSetDevice(ctx->device));
    kfbi_prob3* p = new (std::nothrow) kfbi_prob3;
    if (!p) return set_err(KFBI_ERR_OOM, "host allocation failed");
    p->ctx = ctx;
    p->kappa = d->kappa;
    p->tol = d->tol > 0 ? d->tol : 1e-10;
    p->restart = restart;
    p->max_iter = d->max_iter > 0 ? d->max_iter : 500;
    try {
        p->plan = build_plan3(d->n, d->lo, d->hi, d->axes);
    } catch (const GeometryError& g) {
        delete p;
        return set_err(KFBI_ERR_GEOMETRY, g.msg);
    } catch (const std::bad_alloc&) {
        delete p;
        return set_err(KFBI_ERR_OOM, "host allocation failed in the plan");
    }
    const Plan3Host& P = p->plan;
    const int N = P.N, M = P.M(), I = P.I();
    p->N = N;
    p->M = M;
    p->I = I;
    auto fail = [&](kfbi_status s) {
        free3(p);
        return s;
    };
    DevPlan3& dp = p->dp;
    dp.N = N;
    dp.log2N = 0;
    while ((1 << dp.log2N) < N) ++dp.log2N;
    dp.M = M;
    dp.I = I;
    dp.h = P.h;
    dp.h2 = P.h * P.h;
    dp.kappa = p->kappa;
    std::vector<double> sinq(N / 2 + 1);
    for (int k = 0; k <= N / 2; ++k) sinq[k] = std::sin(M_PI * k / N);
    sinq[N / 2] = 1.0;
    std::vector<ModeConst> modes((size_t)(N - 1) * (N - 1));
    for (int m = 1; m < N; ++m) {
        const double sm = std::sin(M_PI * m / (2.0 * N));
        for (int l = 1; l < N; ++l) {
            const double sl = std::sin(M_PI * l / (2.0 * N));
            modes[(size_t)(m - 1) * (N - 1) + (l - 1)] =
                row_solve_constants(P.h * P.h * p->kappa + 4.0 * sl * sl + 4.0 * sm * sm, N);
        }
    }
    kfbi_status st;
    if ((st = upload3(p, &dp.sinq, sinq)) || (st = upload3(p, &dp.modes, modes)) ||
        (st = upload3(p, &dp.geo, P.geo)) || (st = upload3(p, &dp.fit_off, P.fit_off)) ||
        (st = upload3(p, &dp.fit_idx, P.fit_idx)) || (st = upload3(p, &dp.fit_w, P.fit_w)) ||
        (st = upload3(p, &dp.irr_node, P.irr_node)) || (st = upload3(p, &dp.irr_sign, P.irr_sign)) ||
        (st = upload3(p, &dp.arm_off, P.arm_off)) || (st = upload3(p, &dp.arm_q, P.arm_q)) ||
        (st = upload3(p, &dp.arm_d, P.arm_d)) || (st = upload3(p, &dp.q_axis, P.axis)) ||
        (st = upload3(p, &dp.st_node, P.st_node)) || (st = upload3(p, &dp.st_w, P.st_w)) ||
        (st = upload3(p, &dp.st_t, P.st_t)) || (st = upload3(p, &dp.inside, P.inside)))
        return fail(st);
    const int m = p->restart;
    GmresBufs& b = p->gm;
    if ((st = alloc3(p, &p->G, (size_t)N * N * N)) || (st = alloc3(p, &p->J, (size_t)kJump3 * M)) ||
        (st = alloc3(p, &p->tmpM, M)) || (st = alloc3(p, &p->zeroM, M)) || (st = alloc3(p, &p->d_flag, 1)) ||
        (st = alloc3(p, &b.V, (size_t)(m + 1) * M)) || (st = alloc3(p, &b.H, (size_t)(m + 1) * m)) ||
        (st = alloc3(p, &b.cs, m)) || (st = alloc3(p, &b.sn, m)) || (st = alloc3(p, &b.g, m + 1)) ||
        (st = alloc3(p, &b.ghat, M)) || (st = alloc3(p, &b.phi, M)) || (st = alloc3(p, &b.xcur, M)) ||
        (st = alloc3(p, &b.w, M)) || (st = alloc3(p, &b.z, M)) ||
        (st = alloc3(p, &b.part, gm_part_size(m, gm_chunks(M), gm_chunks64(M)))) || (st = alloc3(p, &b.y, m + 1)) ||
        (st = alloc3(p, &b.st, 1)) || (st = alloc3(p, &b.cnt, 1)))
        return fail(st);
    b.s2cur = nullptr;
    b.m = m;
    b.gc = gm_chunks(M);
    b.gc64 = gm_chunks64(M);
    if (hipMemset(b.cnt, 0, sizeof(unsigned)) != hipSuccess || hipMemset(p->zeroM, 0, M * sizeof(double)) != hipSuccess)
        return fail(set_err(KFBI_ERR_DEVICE, "hipMemset failed"));
    p->dstB = dst_default_tile(N, 2 * sizeof(double), ctx->lds_max, (long)N * N, ctx->num_cu);
    if (p->dstB == 0) return fail(set_err(KFBI_ERR_UNSUPPORTED, "no column-transform tile fits this grid"));
    *out = p;
    return KFBI_OK;
}

kfbi_status kfbi3_prob_destroy(kfbi_prob3* p) {
    if (!p) return KFBI_OK;
    hipSetDevice(p->ctx->device);
    hipStreamSynchronize(p->ctx->stream);
    free3(p);
    return KFBI_OK;
}

kfbi_status kfbi3_prob_info(const kfbi_prob3* p, int* M, int* n_irregular, size_t* device_bytes) {
    if (!p) return set_err(KFBI_ERR_ARG, "prob is NULL");
    if (M) *M = p->M;
    if (n_irregular) *n_irregular = p->I;
    if (device_bytes) *device_bytes = p->bytes;
    return KFBI_OK;
}

kfbi_status kfbi3_prob_points(const kfbi_prob3* p, double* pts, int* axis) {
    if (!p) return set_err(KFBI_ERR_ARG, "prob is NULL");
    if (pts) std::copy(p->plan.pos.begin(), p->plan.pos.end(), pts);
    if (axis) std::copy(p->plan.axis.begin(), p->plan.axis.end(), axis);
    return KFBI_OK;
}

kfbi_status kfbi3_prob_mask(const kfbi_prob3* p, unsigned char* inside) {
    if (!p || !inside) return set_err(KFBI_ERR_ARG, "NULL argument");
    std::copy(p->plan.inside.begin(), p->plan.inside.end(), inside);
    return KFBI_OK;
}

kfbi_status kfbi3_prob_irregular(const kfbi_prob3* p, int* node) {
    if (!p || !node) return set_err(KFBI_ERR_ARG, "NULL argument");
    std::copy(p->plan.irr_node.begin(), p->plan.irr_node.end(), node);
    return KFBI_OK;
}

kfbi_status kfbi3_jumps(kfbi_prob3* p, const double* phi, const double* f_gamma, double* J) {
    if (!p) return set_err(KFBI_ERR_ARG, "prob is NULL");
    if (kfbi_status s = check_ptr(phi, "phi")) return s;
    if (kfbi_status s = check_ptr(J, "J")) return s;
    HIP_TRY(hipSetDevice(p->ctx->device));
    HIP_TRY(launch_jumps3(p->dp, phi, f_gamma, J, nullptr, p->ctx->stream));
    return KFBI_OK;
}

kfbi_status kfbi3_apply(kfbi_prob3* p, const double* phi, double* out) {
    if (!p) return set_err(KFBI_ERR_ARG, "prob is NULL");
    if (kfbi_status s = check_ptr(phi, "phi")) return s;
    if (kfbi_status s = check_ptr(out, "out")) return s;
    HIP_TRY(hipSetDevice(p->ctx->device));
    // the density is checked first; with a NaN or Inf nothing is enqueued
    hipStream_t s = p->ctx->stream;
    HIP_TRY(launch_nonfinite(p->M, phi, p->d_flag, s));
    HIP_TRY(hipMemcpyAsync(&p->h_flag, p->d_flag, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (p->h_flag) return set_err(KFBI_ERR_NONFINITE, "NaN or Inf in the density");
    return interface3(p, phi, nullptr, nullptr, nullptr, false, out);
}

kfbi_status kfbi3_interface_solve(kfbi_prob3* p, const double* phi, const double* f_grid, const double* f_gamma,
                                  double* vgrid, double* vz) {
    if (!p) return set_err(KFBI_ERR_ARG, "prob is NULL");
    if (!vgrid && !vz) return set_err(KFBI_ERR_ARG, "no output requested");
    HIP_TRY(hipSetDevice(p->ctx->device));
    return interface3(p, phi, f_grid, f_gamma, vgrid, false, vz);
}

kfbi_status kfbi3_solve(kfbi_prob3* p, const double* f_grid, const double* f_gamma, const double* g, double* u_grid,
                        double* u_gamma, double* phi, int* iters, double* rel_res) {
    if (!p) return set_err(KFBI_ERR_ARG, "prob is NULL");
    for (auto [ptr, name] : {std::pair<const void*, const char*>{f_grid, "f_grid"}, {f_gamma, "f_gamma"}, {g, "g"},
                             {u_grid, "u_grid"}, {u_gamma, "u_gamma"}, {phi, "phi"}})
        if (kfbi_status s = check_ptr(ptr, name)) return s;
    HIP_TRY(hipSetDevice(p->ctx->device));
    hipStream_t s = p->ctx->stream;
    const int M = p->M;
    // g^ = g - (Y f)^+
    if (kfbi_status e = interface3(p, nullptr, f_grid, f_gamma, nullptr, false, p->tmpM)) return e;
    GmresBufs b = p->gm;
    HIP_TRY(launch_axpby(M, 1.0, g, -1.0, p->tmpM, b.ghat, s));
    GmresState st{};
    if (kfbi_status e = run_gmres3(p, phi, p->tol, p->max_iter, &st)) return e;
    if (st.converged == kGmNonfinite) return set_err(KFBI_ERR_NONFINITE, "NaN or Inf in f, f_gamma, g or phi");
    // u = W phi + Y f
    if (kfbi_status e = interface3(p, b.phi, f_grid, f_gamma, u_grid, true, u_gamma)) return e;
    HIP_TRY(hipMemcpyAsync(phi, b.phi, M * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (iters) *iters = st.it;
    if (rel_res) *rel_res = st.relres;
    if (st.converged == 1) return KFBI_OK;
    return set_err(KFBI_NOT_CONVERGED, "GMRES reached the iteration cap");
}

kfbi_status kfbi3_gmres(kfbi_prob3* p, const double* rhs, double* phi, double tol, int max_iter, int* iters,
                        int* applies, double* rel_res) {
    if (!p) return set_err(KFBI_ERR_ARG, "prob is NULL");
    if (kfbi_status e = check_ptr(rhs, "rhs")) return e;
    if (kfbi_status e = check_ptr(phi, "phi")) return e;
    if (max_iter <= 0) return set_err(KFBI_ERR_ARG, "max_iter must be positive");
    HIP_TRY(hipSetDevice(p->ctx->device));
    hipStream_t s = p->ctx->stream;
    HIP_TRY(hipMemcpyAsync(p->gm.ghat, rhs, p->M * sizeof(double), hipMemcpyDeviceToDevice, s));
    GmresState st{};
    if (kfbi_status e = run_gmres3(p, phi, tol, max_iter, &st)) return e;
    if (st.converged == kGmNonfinite) return set_err(KFBI_ERR_NONFINITE, "NaN or Inf in rhs or the initial guess");
    HIP_TRY(hipMemcpyAsync(phi, p->gm.phi, p->M * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (iters) *iters = st.it;
    if (applies) *applies = st.it + st.res_applies;
    if (rel_res) *rel_res = st.relres;
    if (st.converged == 1) return KFBI_OK;
    return set_err(KFBI_NOT_CONVERGED, "GMRES reached the iteration cap");
}

}  // extern "C"
