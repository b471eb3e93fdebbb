// HIP kernels of the KFBI hot path for gfx950 (MI355X), FP64.
//
// One K_D apply (Sec. 3, Alg. 1 steps 4-6) is three launches:
//   k_correct  one thread per irregular node: jumps at the crossings on its
//              arms (Alg. 2 line 4) and the correction of its right-hand side
//              (Alg. 2 line 5).  For the double-layer apply F = 0, so the
//              right-hand side of the corrected system is nonzero only here.
//   k_modes    the fast solver (Alg. 4) restricted to what the interpolation
//              reads, R sine modes per workgroup.  Along y the right-hand side
//              is expanded in sines; for a sparse right-hand side each
//              coefficient is a short sum over the irregular nodes of one grid
//              column.  Along x each sine mode is a constant-coefficient
//              tridiagonal system, solved by one wavefront as two first-order
//              recurrences (chunked, with wave-wide carry scans) plus a rank-one
//              boundary fix.  The inverse sine sum along y is evaluated only at
//              the six stencil nodes of each boundary sample, already weighted
//              by the interpolation weights, and written as the workgroup's row
//              of partial sums.
//   k_reduce_interp  one wavefront per sample: the partials summed in a fixed
//              order plus the jump terms of the stencil nodes outside Omega
//              (Alg. 3).
// k_spline precomputes the spline second derivatives of the density (inside
// GMRES the emit launch of gmres.h does it for the next input).
// The dense solve (volume potential, final solution) uses the same tridiagonal
// solver on full rows (k_rows_solve), between two column sine transforms
// (dst.hip); in the FP32 mode the transforms and the stored rows are FP32 and
// k_residual forms the FP64 residual of the refinement step.
#include <hip/hip_runtime.h>

#include "device.h"
#include "gmres.h"
#include "graph.h"
#include "kernels.h"

namespace kfbi {

namespace {

// ---------------------------------------------------------------- correction (Alg. 2)

__global__ __launch_bounds__(256) void k_correct(DevPlan p, JumpSrc js, double* __restrict__ corr,
                                                 double* __restrict__ corr_il, double* __restrict__ dense,
                                                 const int* __restrict__ skip) {
    if (skip && *skip) return;
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= p.I) return;
    const double acc = correction_at(p, js, r);
    if (corr) corr[r] = acc;
    if (corr_il) corr_il[p.il_pos[r]] = acc;
    if (dense) dense[(size_t)(p.irr_j[r] - 1) * p.N + (p.irr_i[r] - 1)] += acc;
}

// ---------------------------------------------------------------- sparse fast solve + weighted gather

template <int C, int R>
__global__ __launch_bounds__(kModeWaves * 64) void k_modes(DevPlan p, const double* __restrict__ corr,
                                                          double* __restrict__ partial, const int* __restrict__ skip) {
    extern __shared__ double smem[];
    const ModesLds L = modes_lds<R>(smem, p.N);
    double* row = partial + (size_t)blockIdx.x * p.M;
    modes_round<C, R>(p, corr, blockIdx.x * R, L, [&](int cp, double v) { row[cp] = v; }, p.sinq, skip);
}

// ---------------------------------------------------------------- spline of a density

__global__ __launch_bounds__(256) void k_spline(DevPlan p, const double* __restrict__ y, double* __restrict__ s2,
                                                const int* __restrict__ skip) {
    if (skip && *skip) return;
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m < p.M) s2[m] = spline_s2(y, p.M, p.taps, m);
}

// ---------------------------------------------------------------- interpolation (Alg. 3)

// 64 samples per workgroup of 16 wavefronts (reduce_samples64).
__global__ __launch_bounds__(1024) void k_reduce_interp(DevPlan p, JumpSrc js, const double* __restrict__ partial,
                                                        int G, double* __restrict__ out, const int* __restrict__ skip) {
    __shared__ double red[16 * 64];
    reduce_samples64(p, js, partial, G, blockIdx.x * 64, out, red, skip);
}

// Interpolation from a full grid solution (dense path): R in the padded interior layout.
__global__ __launch_bounds__(256) void k_interp_grid(DevPlan p, JumpSrc js, const double* __restrict__ R,
                                                     double* __restrict__ out) {
    const int cp = blockIdx.x * blockDim.x + threadIdx.x;
    if (cp >= p.M) return;
    int ni[6], nj[6];
    stencil_nodes(p, cp, ni, nj);
    const double* w = p.cp_w + 6 * (size_t)cp;
    double s = 0.0;
    for (int k = 0; k < 6; ++k) s += w[k] * R[(size_t)(nj[k] - 1) * p.N + (ni[k] - 1)];
    out[cp] = s + outside_terms(p, js, cp, ni, nj, w);
}

// ---------------------------------------------------------------- dense path

// R (N x N, interior node (i, j) at (j-1) N + (i-1), row/column N-1 zero pad)
// from a grid array; `mask` keeps only nodes in Omega (the zero extension f~).
__global__ __launch_bounds__(256) void k_fill_rhs(DevPlan p, const double* __restrict__ f, int mask,
                                                  double* __restrict__ R) {
    const int N = p.N;
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)N * N) return;
    const int i = (int)(idx % N) + 1, j = (int)(idx / N) + 1;
    double v = 0.0;
    if (i < N && j < N) {
        const size_t g = (size_t)j * (N + 1) + i;
        v = f ? f[g] : 0.0;
        if (mask && !p.inside[g]) v = 0.0;
    }
    R[idx] = v;
}

// One wavefront per sine mode l (row l-1 of A): the tridiagonal solve along x,
// in FP64 whatever the storage type T.  The solve wants each lane's C
// consecutive values in registers; the row goes through LDS so that the global
// loads and stores stay coalesced (lane-consecutive), one skipped slot per C
// values keeping the lanes' chunk reads on distinct banks.  Rows per
// workgroup: 4 up to C = 16, 2 at C = 32, 1 at C = 64 (33.8 KB of LDS).
template <int C>
constexpr int rows_per_group() { return C <= 16 ? 4 : C == 32 ? 2 : 1; }

template <int C, class T>
__global__ __launch_bounds__(64 * rows_per_group<C>()) void k_rows_solve(DevPlan p, T* __restrict__ A) {
    constexpr int RPW = rows_per_group<C>(), W = 64 * C, WP = W + 64;
    __shared__ double rs[RPW][WP];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int l = blockIdx.x * RPW + w + 1;
    const bool live = l <= p.n;                          // the barriers below are the workgroup's
    T* row = A + (size_t)(l - 1) * p.N;
    double* r = rs[w];
    auto pad = [](int e) { return e + e / C; };
    if (live) {
#pragma unroll 8
        for (int c = 0; c < C; ++c) r[pad(c * 64 + lane)] = (double)row[c * 64 + lane] * p.h2;
    }
    __syncthreads();
    double e[C];
    if (live) {
#pragma unroll
        for (int c = 0; c < C; ++c) e[c] = r[pad(lane * C + c)];
        mode_solve<C>(e, p.modes[l], lane, p.N);
#pragma unroll
        for (int c = 0; c < C; ++c) r[pad(lane * C + c)] = e[c];
    }
    __syncthreads();
    if (live) {
#pragma unroll 8
        for (int c = 0; c < C; ++c) row[c * 64 + lane] = (T)r[pad(c * 64 + lane)];
    }
}

// R <- R - ((V_E + V_W + V_N + V_S - 4 V) / h^2 - kappa V) at the interior nodes
// (V = 0 on the box), all in the padded interior layout; with A, also A <- A + V.
__global__ __launch_bounds__(256) void k_residual(DevPlan p, const double* __restrict__ V, double* __restrict__ R,
                                                  double* __restrict__ A) {
    const int N = p.N;
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)N * N) return;
    const int i = (int)(idx % N) + 1, j = (int)(idx / N) + 1;
    if (i >= N || j >= N) return;
    const double v = V[idx];
    const double vw = i > 1 ? V[idx - 1] : 0.0;
    const double ve = i < N - 1 ? V[idx + 1] : 0.0;
    const double vs = j > 1 ? V[idx - N] : 0.0;
    const double vn = j < N - 1 ? V[idx + N] : 0.0;
    R[idx] -= (vw + ve + vs + vn - 4.0 * v) * p.inv_h2 - p.kappa * v;
    if (A) A[idx] += v;
}

__global__ __launch_bounds__(256) void k_grid_out(DevPlan p, const double* __restrict__ R, int mask,
                                                  double* __restrict__ u) {
    const int W1 = p.N + 1;
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)W1 * W1) return;
    const int i = (int)(idx % W1), j = (int)(idx / W1);
    double v = 0.0;
    if (i >= 1 && j >= 1 && i <= p.n && j <= p.n) v = R[(size_t)(j - 1) * p.N + (i - 1)];
    if (mask && !p.inside[idx]) v = 0.0;
    u[idx] = v;
}

__global__ __launch_bounds__(256) void k_axpby(int n, double a, const double* __restrict__ x, double b,
                                               const double* __restrict__ y, double* __restrict__ z) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) z[i] = a * x[i] + (y ? b * y[i] : 0.0);
}

__global__ __launch_bounds__(256) void k_fill(size_t n, double v, double* __restrict__ x) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = v;
}

// flag <- 1 if any of x[0..n) is NaN or Inf, else 0: one workgroup, which
// writes the flag whatever it finds (nothing to clear beforehand)
__global__ __launch_bounds__(256) void k_nonfinite(int n, const double* __restrict__ x, int* __restrict__ flag) {
    __shared__ int any;
    if (threadIdx.x == 0) any = 0;
    __syncthreads();
    int bad = 0;
    for (int i = threadIdx.x; i < n; i += 256) bad |= !isfinite(x[i]);
    if (bad) any = 1;                                    // benign race: every writer stores 1
    __syncthreads();
    if (threadIdx.x == 0) *flag = any;
}

// ---------------------------------------------------------------- GMRES step (Alg. 5)

// the apply's last launch inside GMRES: w at 64 samples, then the first pass
__global__ __launch_bounds__(1024) void k_reduce_gm(DevPlan p, JumpSrc js, const double* __restrict__ partial, int G,
                                                    GmresBufs b) {
    __shared__ double red[16 * 64];
    const GmPre pre = gm_dots1_prefetch(b, p.M, blockIdx.x);
    const int mode = load_flag_late(&b.st->mode), j = load_flag_late(&b.st->j);   // waited for where used
    if (!reduce_samples64(p, js, partial, G, blockIdx.x * 64, b.w, red, &b.st->converged)) return;
    gm_dots1_64(b, p.M, blockIdx.x, red, &pre, mode, j);
}
__global__ __launch_bounds__(kGmChunk) void k_gm_upd1(GmresBufs b, int M) { gm_update1_commit(b, M, blockIdx.x); }
__global__ __launch_bounds__(kGmChunk) void k_gm_begin(DevPlan p, int has_p, const double* taps, GmresBufs b, int M,
                                                       const double* rhs, const double* phi_in, double tol,
                                                       int max_iter, double reorth, double* xout, double* corr_il) {
    gm_begin(has_p ? &p : nullptr, taps, b, M, rhs, phi_in, tol, max_iter, reorth, xout, corr_il);
}
__global__ __launch_bounds__(kGmChunk) void k_gm_emit(const double* taps, GmresBufs b, int M) {
    gm_emit(taps, b, M, blockIdx.x);
}
// the emit launch with the next apply's corrections: workgroups 0 .. gc-1
// emit, the rest make one correction chunk each
__global__ __launch_bounds__(kGmChunk) void k_gm_emit_corr(DevPlan p, GmresBufs b, double* __restrict__ corr_il) {
    if ((int)blockIdx.x < b.gc) {
        gm_emit(p.taps, b, p.M, blockIdx.x);
    } else {
        gm_emit_corrections(p, b, (int)blockIdx.x - b.gc, corr_il);
    }
}


template <int C, int R>
hipError_t modes_launch(const DevPlan& p, const double* corr, double* partial, const int* skip, hipStream_t s) {
    constexpr size_t lds = sizeof(double) * ((size_t)(32 * C + 2) + (size_t)R * (64 * (C + 1) + kMaxExtra));
    if constexpr (lds > 160 * 1024) {
        return hipErrorInvalidValue;                  // never fits the local data share
    } else {
        if (hipError_t e = hipFuncSetAttribute((const void*)k_modes<C, R>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                               (int)lds))
            return e;
        const int groups = (p.n + R - 1) / R;
        return klaunch(&k_modes<C, R>, dim3(groups), dim3(kModeWaves * 64), lds, s, p, corr, partial, skip);
    }
}

template <int C>
hipError_t modes_dispatch_r(const DevPlan& p, const double* corr, double* partial, int R, const int* skip,
                            hipStream_t s) {
    switch (R) {
        case 1: return modes_launch<C, 1>(p, corr, partial, skip, s);
        case 2: return modes_launch<C, 2>(p, corr, partial, skip, s);
        case 4: return modes_launch<C, 4>(p, corr, partial, skip, s);
        case 8: return modes_launch<C, 8>(p, corr, partial, skip, s);
        default: return hipErrorInvalidValue;
    }
}

template <int C, class T>
hipError_t rows_dispatch(const DevPlan& p, T* A, hipStream_t s) {
    constexpr int RPW = rows_per_group<C>();
    if (hipError_t e_ = klaunch(&k_rows_solve<C, T>, dim3((p.n + RPW - 1) / RPW), dim3(64 * RPW), 0, s, p, A))
        return e_;
    return hipGetLastError();
}

template <class T>
hipError_t rows_solve_any(const DevPlan& p, T* A, hipStream_t s) {
    switch (p.N) {
        case 64: return rows_dispatch<1>(p, A, s);
        case 128: return rows_dispatch<2>(p, A, s);
        case 256: return rows_dispatch<4>(p, A, s);
        case 512: return rows_dispatch<8>(p, A, s);
        case 1024: return rows_dispatch<16>(p, A, s);
        case 2048: return rows_dispatch<32>(p, A, s);
        case 4096: return rows_dispatch<64>(p, A, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

size_t modes_lds_bytes(int N, int R) {
    return sizeof(double) * ((size_t)(N / 2 + 2) + (size_t)R * (N + 64 + kMaxExtra));
}

hipError_t launch_correct(const DevPlan& p, JumpSrc js, double* corr, double* corr_il, double* dense,
                          const int* skip, hipStream_t s) {
    if (p.I == 0) return hipSuccess;
    if (hipError_t e_ = klaunch(&k_correct, dim3((p.I + 255) / 256), dim3(256), 0, s, p, js, corr, corr_il, dense, skip)) return e_;
    return hipGetLastError();
}

hipError_t launch_modes(const DevPlan& p, const double* corr, double* partial, int R, const int* skip,
                        hipStream_t s) {
    switch (p.N) {
        case 64: return modes_dispatch_r<1>(p, corr, partial, R, skip, s);
        case 128: return modes_dispatch_r<2>(p, corr, partial, R, skip, s);
        case 256: return modes_dispatch_r<4>(p, corr, partial, R, skip, s);
        case 512: return modes_dispatch_r<8>(p, corr, partial, R, skip, s);
        case 1024: return modes_dispatch_r<16>(p, corr, partial, R, skip, s);
        case 2048: return modes_dispatch_r<32>(p, corr, partial, R, skip, s);
        case 4096: return modes_dispatch_r<64>(p, corr, partial, R, skip, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_spline(const DevPlan& p, const double* y, double* s2, const int* skip, hipStream_t s) {
    if (hipError_t e_ = klaunch(&k_spline, dim3((p.M + 255) / 256), dim3(256), 0, s, p, y, s2, skip)) return e_;
    return hipGetLastError();
}

hipError_t launch_reduce_interp(const DevPlan& p, JumpSrc js, const double* partial, int G, double* out,
                                const int* skip, const GmresBufs* gm, hipStream_t s) {
    if (gm) return klaunch(&k_reduce_gm, dim3((p.M + 63) / 64), dim3(1024), 0, s, p, js, partial, G, *gm);
    if (hipError_t e_ = klaunch(&k_reduce_interp, dim3((p.M + 63) / 64), dim3(1024), 0, s, p, js, partial, G, out, skip)) return e_;
    return hipGetLastError();
}

hipError_t launch_interp_grid(const DevPlan& p, JumpSrc js, const double* R, double* out, hipStream_t s) {
    if (hipError_t e_ = klaunch(&k_interp_grid, dim3((p.M + 255) / 256), dim3(256), 0, s, p, js, R, out)) return e_;
    return hipGetLastError();
}

hipError_t launch_fill_rhs(const DevPlan& p, const double* f, bool mask, double* R, hipStream_t s) {
    const size_t tot = (size_t)p.N * p.N;
    if (hipError_t e_ = klaunch(&k_fill_rhs, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, p, f, mask ? 1 : 0, R)) return e_;
    return hipGetLastError();
}

hipError_t launch_rows_solve(const DevPlan& p, double* A, hipStream_t s) { return rows_solve_any(p, A, s); }

hipError_t launch_rows_solve_f32(const DevPlan& p, float* A, hipStream_t s) { return rows_solve_any(p, A, s); }

hipError_t launch_residual(const DevPlan& p, const double* V, double* R, double* A, hipStream_t s) {
    const size_t tot = (size_t)p.N * p.N;
    if (hipError_t e_ = klaunch(&k_residual, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, p, V, R, A)) return e_;
    return hipGetLastError();
}

hipError_t launch_grid_out(const DevPlan& p, const double* R, bool mask, double* u, hipStream_t s) {
    const size_t tot = (size_t)(p.N + 1) * (p.N + 1);
    if (hipError_t e_ = klaunch(&k_grid_out, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, p, R, mask ? 1 : 0, u)) return e_;
    return hipGetLastError();
}

hipError_t launch_axpby(int n, double a, const double* x, double b, const double* y, double* z, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (hipError_t e_ = klaunch(&k_axpby, dim3((n + 255) / 256), dim3(256), 0, s, n, a, x, b, y, z)) return e_;
    return hipGetLastError();
}

hipError_t launch_fill(size_t n, double v, double* x, hipStream_t s) {
    if (n == 0) return hipSuccess;
    if (hipError_t e_ = klaunch(&k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, v, x)) return e_;
    return hipGetLastError();
}

hipError_t launch_nonfinite(int n, const double* x, int* flag, hipStream_t s) {
    if (hipError_t e_ = klaunch(&k_nonfinite, dim3(1), dim3(256), 0, s, n, x, flag)) return e_;
    return hipGetLastError();
}

hipError_t launch_gmres_step_corr(const DevPlan& p, GmresBufs b, double* corr_il, hipStream_t s) {
    const dim3 g(b.gc), t(kGmChunk);
    if (hipError_t e = klaunch(&k_gm_upd1, g, t, 0, s, b, p.M)) return e;
    return klaunch(&k_gm_emit_corr, dim3(b.gc + p.n_cc), t, 0, s, p, b, corr_il);
}

hipError_t launch_gmres_start(const DevPlan* p, const double* taps, int M, GmresBufs b, const double* rhs,
                              const double* phi_in, double tol, int max_iter, double reorth, double* xout,
                              double* corr_il, hipStream_t s) {
    const bool corr = p && corr_il;
    const DevPlan pv = corr ? *p : DevPlan{};
    const int groups = b.gc + (corr ? p->n_cc : 0);
    return klaunch(&k_gm_begin, dim3(groups), dim3(kGmChunk), 0, s, pv, corr ? 1 : 0, taps, b, M, rhs, phi_in, tol,
                   max_iter, reorth, xout, corr ? corr_il : nullptr);
}

hipError_t launch_gmres_step(const double* taps, int M, GmresBufs b, hipStream_t s) {
    const dim3 g(b.gc), t(kGmChunk);
    if (hipError_t e = klaunch(&k_gm_upd1, g, t, 0, s, b, M)) return e;
    return klaunch(&k_gm_emit, g, t, 0, s, taps, b, M);
}

}  // namespace kfbi
