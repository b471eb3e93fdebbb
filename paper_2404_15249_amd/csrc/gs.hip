// Gray-Scott reaction-diffusion by Strang splitting (Example 3) on the
// Neumann solve of this library.
//
// One step is R(dt/2) D(dt) R(dt/2):
//  - R: the pointwise reaction ODE u' = (gamma (1-u) - u v^2)/eps0,
//    v' = (u v^2 - (gamma + kill) v)/eps0, one classical Runge-Kutta step of
//    dt/2, at the grid nodes in Omega and at the boundary samples (the state
//    keeps its trace on Gamma: the diffusion solve needs it as the jump [F]);
//  - D: Crank-Nicolson for w' = eps Lap w with d_n w = 0, as w <- 2 z - w with
//    z the backward-Euler half step Lap z - kappa z = -kappa w, kappa = 2/(eps dt):
//    one Neumann solve per species, warm-started from the species' previous
//    density.  The two species' solves are independent: each problem has its
//    own stream and the solves overlap (solve_neumann_pair).
//    The half step is solved as z = c + z', c the mean of w's trace at the
//    samples: Lap z' - kappa z' = -kappa (w - c), d_n z' = 0.  A constant solves
//    the Neumann problem exactly, so this is the same z; but the zero extension
//    of the right-hand side outside Omega (the volume potential of the Sec. 2.2
//    table) then jumps across Gamma by kappa (w - c), not kappa w, which at
//    kappa h^2 of order one would otherwise lift a uniform state near Gamma.
// Grid nodes outside Omega hold zero.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "api_common.h"

using namespace kfbi;

namespace {

struct GsRates {
    double gamma, kill, inv_eps0;
};

__device__ __forceinline__ void gs_rates(double u, double v, const GsRates& P, double& du, double& dv) {
    const double uvv = u * v * v;
    du = (P.gamma * (1.0 - u) - uvv) * P.inv_eps0;
    dv = (uvv - (P.gamma + P.kill) * v) * P.inv_eps0;
}

// One classical RK4 step of size dt.
__device__ __forceinline__ void gs_rk4(double& u, double& v, double dt, const GsRates& P) {
    double a1, b1, a2, b2, a3, b3, a4, b4;
    gs_rates(u, v, P, a1, b1);
    gs_rates(u + 0.5 * dt * a1, v + 0.5 * dt * b1, P, a2, b2);
    gs_rates(u + 0.5 * dt * a2, v + 0.5 * dt * b2, P, a3, b3);
    gs_rates(u + dt * a3, v + dt * b3, P, a4, b4);
    const double c = dt / 6.0;
    u = u + c * (a1 + 2.0 * a2 + 2.0 * a3 + a4);
    v = v + c * (b1 + 2.0 * b2 + 2.0 * b3 + b4);
}

// Element t of the state: grid node t (t < ng, kept only where mask is set) or
// boundary sample t - ng.
struct GsState {
    double* u;      // ng, then the M samples (one buffer: grid followed by trace)
    double* v;
    const unsigned char* mask;   // ng
    int ng, M;
};

constexpr int kMeanThreads = 256;

// The means c_u, c_v of the two species' traces after R(dt/2): one workgroup
// applies the reaction half step to the M trace values itself (the same
// pointwise step k_gs_pre makes) and sums them in a fixed order.
__global__ __launch_bounds__(kMeanThreads) void k_gs_trace_mean(GsState S, double dth, GsRates P,
                                                                double* __restrict__ cmean) {
    __shared__ double su[kMeanThreads], sv[kMeanThreads];
    const int tid = threadIdx.x;
    double a = 0.0, b = 0.0;
    for (int t = tid; t < S.M; t += kMeanThreads) {
        double u = S.u[S.ng + t], v = S.v[S.ng + t];
        gs_rk4(u, v, dth, P);
        a += u;
        b += v;
    }
    su[tid] = a;
    sv[tid] = b;
    __syncthreads();
    for (int w = kMeanThreads / 2; w > 0; w >>= 1) {
        if (tid < w) {
            su[tid] += su[tid + w];
            sv[tid] += sv[tid + w];
        }
        __syncthreads();
    }
    if (tid == 0) {
        cmean[0] = su[0] / S.M;
        cmean[1] = sv[0] / S.M;
    }
}

// R(dt/2), then the right-hand sides of the two half-step solves for z' = z - c:
// fu = -kappa_u (u - c_u), fv = -kappa_v (v - c_v) in Omega and at the samples,
// zero at the grid nodes outside Omega (same layout as the state).
__global__ __launch_bounds__(256) void k_gs_pre(GsState S, double* __restrict__ fu, double* __restrict__ fv,
                                                double dth, double ku, double kv, GsRates P,
                                                const double* __restrict__ cmean) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= S.ng + S.M) return;
    double u = 0.0, v = 0.0, ru = 0.0, rv = 0.0;
    if (t >= S.ng || S.mask[t]) {
        u = S.u[t];
        v = S.v[t];
        gs_rk4(u, v, dth, P);
        ru = -ku * (u - cmean[0]);
        rv = -kv * (v - cmean[1]);
    }
    S.u[t] = u;
    S.v[t] = v;
    fu[t] = ru;
    fv[t] = rv;
}

// w <- 2 (c + z') - w for both species (z' from the solves: grid zero outside
// Omega, then the trace), then R(dt/2).
__global__ __launch_bounds__(256) void k_gs_post(GsState S, const double* __restrict__ zu,
                                                 const double* __restrict__ zv, double dth, GsRates P,
                                                 const double* __restrict__ cmean) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= S.ng + S.M) return;
    double u = 0.0, v = 0.0;
    if (t >= S.ng || S.mask[t]) {
        u = 2.0 * (cmean[0] + zu[t]) - S.u[t];
        v = 2.0 * (cmean[1] + zv[t]) - S.v[t];
        gs_rk4(u, v, dth, P);
    }
    S.u[t] = u;
    S.v[t] = v;
}

}  // namespace

struct kfbi_gs {
    kfbi_ctx* ctx = nullptr;     // the caller's context: stream A (state, pointwise kernels, u)
    kfbi_ctx* ctx2 = nullptr;    // the second stream (v's solve)
    hipEvent_t ev_pre = nullptr, ev_solved = nullptr;
    kfbi_prob* pu = nullptr;     // kappa_u = 2/(eps1 dt)
    kfbi_prob* pv = nullptr;     // kappa_v = 2/(eps2 dt)
    kfbi_gs_desc d{};
    int n = 0, M = 0, ng = 0;
    double ku = 0, kv = 0;
    // device buffers; grid arrays are followed by the M trace values
    double *u = nullptr, *v = nullptr, *fu = nullptr, *fv = nullptr, *zu = nullptr, *zv = nullptr;
    double *psi_u = nullptr, *psi_v = nullptr, *gn = nullptr, *dn = nullptr;
    double* cmean = nullptr;     // 2: the trace means c_u, c_v of the current step
    unsigned char* mask = nullptr;
    std::vector<void*> allocs;
    long long iters = 0;         // GMRES iterations of all solves so far
    int steps = 0;
};

namespace {

void gs_free(kfbi_gs* g) {
    // both streams drained (destroying a problem waits for its stream) before
    // the state buffers go
    if (g->pu) kfbi_prob_destroy(g->pu);
    if (g->pv) kfbi_prob_destroy(g->pv);
    g->pu = g->pv = nullptr;
    if (g->ctx2) hipStreamSynchronize(g->ctx2->stream);
    for (void* a : g->allocs) hipFree(a);
    g->allocs.clear();
    if (g->ev_pre) hipEventDestroy(g->ev_pre);
    if (g->ev_solved) hipEventDestroy(g->ev_solved);
    g->ev_pre = g->ev_solved = nullptr;
    if (g->ctx2) kfbi_ctx_destroy(g->ctx2);
    g->ctx2 = nullptr;
}

template <class T>
kfbi_status gs_alloc(kfbi_gs* g, T** out, size_t count) {
    void* p = nullptr;
    if (hipMalloc(&p, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess) {
        hipGetLastError();
        return set_err(KFBI_ERR_OOM, "device allocation failed (Gray-Scott state)");
    }
    g->allocs.push_back(p);
    *out = static_cast<T*>(p);
    return KFBI_OK;
}

}  // namespace

extern "C" {

kfbi_status kfbi_gs_create(kfbi_ctx* ctx, const kfbi_gs_desc* d, kfbi_gs** out) {
    if (!ctx || !d || !out) return set_err(KFBI_ERR_ARG, "NULL argument");
    *out = nullptr;
    if (!(d->dt > 0.0) || !(d->eps0 > 0.0) || !(d->eps1 > 0.0) || !(d->eps2 > 0.0))
        return set_err(KFBI_ERR_ARG, "dt, eps0, eps1 and eps2 must be positive");
    HIP_TRY(hipSetDevice(ctx->device));
    kfbi_gs* g = new kfbi_gs;
    g->ctx = ctx;
    g->d = *d;
    g->d.xy = nullptr;                       // host memory of the caller: not kept
    g->ku = 2.0 / (d->eps1 * d->dt);
    g->kv = 2.0 / (d->eps2 * d->dt);
    auto fail = [&](kfbi_status s) {
        gs_free(g);
        delete g;
        return s;
    };
    kfbi_desc pd{};
    pd.lo = d->lo;
    pd.hi = d->hi;
    pd.n = d->n;
    pd.m = d->m;
    pd.xy = d->xy;
    pd.tol = d->tol;
    pd.restart = d->restart;
    pd.max_iter = d->max_iter;
    pd.precision = KFBI_FP64;
    pd.kappa = g->ku;
    if (kfbi_status s = kfbi_prob_create(ctx, &pd, &g->pu)) return fail(s);
    if (kfbi_status s = kfbi_ctx_create(ctx->device, nullptr, &g->ctx2)) return fail(s);
    pd.kappa = g->kv;
    if (kfbi_status s = kfbi_prob_create(g->ctx2, &pd, &g->pv)) return fail(s);
    if (hipEventCreateWithFlags(&g->ev_pre, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&g->ev_solved, hipEventDisableTiming) != hipSuccess) {
        hipGetLastError();
        return fail(set_err(KFBI_ERR_DEVICE, "event creation failed"));
    }
    kfbi_prob_info(g->pu, &g->M, nullptr, nullptr, nullptr);
    g->n = d->n;
    g->ng = (d->n + 1) * (d->n + 1);
    const size_t all = (size_t)g->ng + g->M;
    kfbi_status st = KFBI_OK;
    if ((st = gs_alloc(g, &g->u, all)) || (st = gs_alloc(g, &g->v, all)) || (st = gs_alloc(g, &g->fu, all)) ||
        (st = gs_alloc(g, &g->fv, all)) || (st = gs_alloc(g, &g->zu, all)) || (st = gs_alloc(g, &g->zv, all)) ||
        (st = gs_alloc(g, &g->psi_u, g->M)) || (st = gs_alloc(g, &g->psi_v, g->M)) ||
        (st = gs_alloc(g, &g->gn, g->M)) || (st = gs_alloc(g, &g->dn, 2 * (size_t)g->M)) ||
        (st = gs_alloc(g, &g->cmean, 2)) || (st = gs_alloc(g, &g->mask, g->ng)))
        return fail(st);
    std::vector<unsigned char> mask(g->ng);
    kfbi_prob_mask(g->pu, mask.data());
    hipStream_t s = ctx->stream;
    if (hipMemcpyAsync(g->mask, mask.data(), g->ng, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemsetAsync(g->u, 0, all * sizeof(double), s) != hipSuccess ||
        hipMemsetAsync(g->v, 0, all * sizeof(double), s) != hipSuccess ||
        hipMemsetAsync(g->psi_u, 0, g->M * sizeof(double), s) != hipSuccess ||
        hipMemsetAsync(g->psi_v, 0, g->M * sizeof(double), s) != hipSuccess ||
        hipMemsetAsync(g->gn, 0, g->M * sizeof(double), s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
        hipGetLastError();
        return fail(set_err(KFBI_ERR_DEVICE, "Gray-Scott state initialisation failed"));
    }
    *out = g;
    return KFBI_OK;
}

kfbi_status kfbi_gs_destroy(kfbi_gs* g) {
    if (!g) return KFBI_OK;
    hipSetDevice(g->ctx->device);
    hipStreamSynchronize(g->ctx->stream);
    gs_free(g);
    delete g;
    return KFBI_OK;
}

kfbi_status kfbi_gs_info(const kfbi_gs* g, int* m, int* steps, long long* gmres_iters) {
    if (!g) return set_err(KFBI_ERR_ARG, "gs is NULL");
    if (m) *m = g->M;
    if (steps) *steps = g->steps;
    if (gmres_iters) *gmres_iters = g->iters;
    return KFBI_OK;
}

kfbi_status kfbi_gs_set_state(kfbi_gs* g, const double* u_grid, const double* v_grid, const double* u_gamma,
                              const double* v_gamma) {
    if (!g) return set_err(KFBI_ERR_ARG, "gs is NULL");
    for (auto [p, name] : {std::pair<const void*, const char*>{u_grid, "u_grid"}, {v_grid, "v_grid"},
                           {u_gamma, "u_gamma"}, {v_gamma, "v_gamma"}})
        if (kfbi_status s = check_ptr(p, name)) return s;
    HIP_TRY(hipSetDevice(g->ctx->device));
    hipStream_t s = g->ctx->stream;
    const size_t gb = (size_t)g->ng * sizeof(double), mb = (size_t)g->M * sizeof(double);
    HIP_TRY(hipMemcpyAsync(g->u, u_grid, gb, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(g->v, v_grid, gb, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(g->u + g->ng, u_gamma, mb, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(g->v + g->ng, v_gamma, mb, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemsetAsync(g->psi_u, 0, mb, s));
    HIP_TRY(hipMemsetAsync(g->psi_v, 0, mb, s));
    g->steps = 0;
    g->iters = 0;
    return KFBI_OK;
}

kfbi_status kfbi_gs_get_state(kfbi_gs* g, double* u_grid, double* v_grid, double* u_gamma, double* v_gamma) {
    if (!g) return set_err(KFBI_ERR_ARG, "gs is NULL");
    HIP_TRY(hipSetDevice(g->ctx->device));
    hipStream_t s = g->ctx->stream;
    const size_t gb = (size_t)g->ng * sizeof(double), mb = (size_t)g->M * sizeof(double);
    if (u_grid) HIP_TRY(hipMemcpyAsync(u_grid, g->u, gb, hipMemcpyDeviceToDevice, s));
    if (v_grid) HIP_TRY(hipMemcpyAsync(v_grid, g->v, gb, hipMemcpyDeviceToDevice, s));
    if (u_gamma) HIP_TRY(hipMemcpyAsync(u_gamma, g->u + g->ng, mb, hipMemcpyDeviceToDevice, s));
    if (v_gamma) HIP_TRY(hipMemcpyAsync(v_gamma, g->v + g->ng, mb, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    return KFBI_OK;
}

kfbi_status kfbi_gs_step(kfbi_gs* g, int nsteps) {
    if (!g) return set_err(KFBI_ERR_ARG, "gs is NULL");
    if (nsteps < 0) return set_err(KFBI_ERR_ARG, "nsteps must be >= 0");
    HIP_TRY(hipSetDevice(g->ctx->device));
    hipStream_t s = g->ctx->stream;
    const GsRates P{g->d.gamma, g->d.kill, 1.0 / g->d.eps0};
    const GsState S{g->u, g->v, g->mask, g->ng, g->M};
    const int total = g->ng + g->M;
    const dim3 grid((total + 255) / 256), block(256);
    const double dth = 0.5 * g->d.dt;
    hipStream_t s2 = g->ctx2->stream;
    const NeumannIO iu{g->fu, g->fu + g->ng, g->gn, g->zu, g->zu + g->ng, g->dn, g->psi_u};
    const NeumannIO iv{g->fv, g->fv + g->ng, g->gn, g->zv, g->zv + g->ng, g->dn + g->M, g->psi_v};
    for (int k = 0; k < nsteps; ++k) {
        HIP_TRY(klaunch(k_gs_trace_mean, dim3(1), dim3(kMeanThreads), 0, s, S, dth, P, g->cmean));
        HIP_TRY(klaunch(k_gs_pre, grid, block, 0, s, S, g->fu, g->fv, dth, g->ku, g->kv, P,
                        (const double*)g->cmean));
        HIP_TRY(hipEventRecord(g->ev_pre, s));             // v's solve reads what k_gs_pre wrote
        HIP_TRY(hipStreamWaitEvent(s2, g->ev_pre, 0));
        int itu = 0, itv = 0;
        if (kfbi_status e = solve_neumann_pair(g->pu, iu, g->pv, iv, &itu, &itv)) return e;
        g->iters += itu + itv;
        HIP_TRY(hipEventRecord(g->ev_solved, s2));         // k_gs_post reads v's solution
        HIP_TRY(hipStreamWaitEvent(s, g->ev_solved, 0));
        HIP_TRY(klaunch(k_gs_post, grid, block, 0, s, S, g->zu, g->zv, dth, P, (const double*)g->cmean));
        g->steps++;
    }
    HIP_TRY(hipStreamSynchronize(s));
    return KFBI_OK;
}

}  // extern "C"
