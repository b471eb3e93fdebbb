// Kernels of the three-dimensional problem (k3.h): the steps of Alg. 1 on the
// 7-point grid around an ellipsoid.
//   k_jumps3    eight lanes per control point: surface derivatives of the
//               density from its fit neighbours (a fixed weighted sum), then
//               the Cartesian jumps from the local frame and shape operator.
//   k_fill3     the base right-hand side in the interior layout.
//   k_correct3  one thread per irregular node: the Taylor-corrected jumps of
//               its arms (Alg. 2), added to the right-hand side.
//   k_rows3     one wavefront per (z-mode, y-mode) row: the tridiagonal
//               solve along x (chunked recurrences, as in two dimensions).
//   k_interp3   the ten-node quadratic interpolation (Alg. 3) as fixed
//               weights, plus the jump terms of far-side nodes.
// The sine transforms along z and y are the column transforms of dst.hip,
// applied to the planes of the grid.
#include <hip/hip_runtime.h>

#include "device.h"
#include "gmres.h"
#include "graph.h"
#include "k3.h"
#include "plan3.h"

namespace kfbi {

namespace {

constexpr int kFitLanes = 8;   // lanes sharing one control point's neighbour sum

__global__ __launch_bounds__(256) void k_jumps3(DevPlan3 p, const double* __restrict__ phi,
                                                const double* __restrict__ fgam, double* __restrict__ J,
                                                const int* __restrict__ skip) {
    if (skip && *skip) return;
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    const int m = gid / kFitLanes, sub = gid % kFitLanes;
    const int M = p.M;
    const bool valid = m < M;
    const double ph = valid ? phi[m] : 0.0;
    // the surface derivatives: each of the point's kFitLanes lanes takes every
    // kFitLanes-th neighbour, then the lanes' sums are combined (fixed order)
    double d0 = 0.0, d1 = 0.0, d2 = 0.0, d3 = 0.0, d4 = 0.0;
    if (valid) {
        for (int e = p.fit_off[m] + sub, e1 = p.fit_off[m + 1]; e < e1; e += kFitLanes) {
            const double dv = phi[p.fit_idx[e]] - ph;
            const double* w = p.fit_w + 5 * (size_t)e;
            d0 = fma(w[0], dv, d0);
            d1 = fma(w[1], dv, d1);
            d2 = fma(w[2], dv, d2);
            d3 = fma(w[3], dv, d3);
            d4 = fma(w[4], dv, d4);
        }
    }
#pragma unroll
    for (int off = kFitLanes / 2; off >= 1; off >>= 1) {
        d0 += __shfl_xor(d0, off, 64);
        d1 += __shfl_xor(d1, off, 64);
        d2 += __shfl_xor(d2, off, 64);
        d3 += __shfl_xor(d3, off, 64);
        d4 += __shfl_xor(d4, off, 64);
    }
    if (!valid || sub != 0) return;
    const double* g = p.geo + 12 * (size_t)m;
    const double nx = g[0], ny = g[1], nz = g[2];
    const double ax = g[3], ay = g[4], az = g[5];     // t1
    const double bx = g[6], by = g[7], bz = g[8];     // t2
    const double s11 = g[9], s12 = g[10], s22 = g[11];
    // tangential block, mixed (tangent, normal) entries, normal-normal entry
    const double h11 = d2, h12 = d3, h22 = d4;
    const double h1n = -(s11 * d0 + s12 * d1);
    const double h2n = -(s12 * d0 + s22 * d1);
    const double F = fgam ? fgam[m] : 0.0;
    const double hnn = F + p.kappa * ph - h11 - h22;
    auto H = [&](double ui, double uj, double vi, double vj, double ni, double nj) {
        return h11 * ui * uj + h22 * vi * vj + h12 * (ui * vj + vi * uj) + h1n * (ui * nj + ni * uj) +
               h2n * (vi * nj + ni * vj) + hnn * ni * nj;
    };
    J[m] = ph;
    J[(size_t)1 * M + m] = d0 * ax + d1 * bx;
    J[(size_t)2 * M + m] = d0 * ay + d1 * by;
    J[(size_t)3 * M + m] = d0 * az + d1 * bz;
    J[(size_t)4 * M + m] = H(ax, ax, bx, bx, nx, nx);
    J[(size_t)5 * M + m] = H(ay, ay, by, by, ny, ny);
    J[(size_t)6 * M + m] = H(az, az, bz, bz, nz, nz);
    J[(size_t)7 * M + m] = H(ax, ay, bx, by, nx, ny);
    J[(size_t)8 * M + m] = H(ax, az, bx, bz, nx, nz);
    J[(size_t)9 * M + m] = H(ay, az, by, bz, ny, nz);
}

__global__ __launch_bounds__(256) void k_fill3(DevPlan3 p, const double* __restrict__ f, double* __restrict__ G,
                                               const int* __restrict__ skip) {
    if (skip && *skip) return;
    const int N = p.N;
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)N * N * N) return;
    const int i = (int)(idx % N) + 1, j = (int)((idx / N) % N) + 1, k = (int)(idx / ((size_t)N * N)) + 1;
    double v = 0.0;
    if (f && i < N && j < N && k < N) {
        const size_t g = ((size_t)k * (N + 1) + j) * (N + 1) + i;
        if (p.inside[g]) v = f[g];
    }
    G[idx] = v;
}

__global__ __launch_bounds__(256) void k_correct3(DevPlan3 p, const double* __restrict__ J, double* __restrict__ G,
                                                  const int* __restrict__ skip) {
    if (skip && *skip) return;
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= p.I) return;
    const int M = p.M;
    const double s = p.irr_sign[r];
    double acc = 0.0;
    for (int a = p.arm_off[r], a1 = p.arm_off[r + 1]; a < a1; ++a) {
        const int q = p.arm_q[a], ax = p.q_axis[q];
        const double d = p.arm_d[a];
        const double jv = J[q] + d * J[(size_t)(1 + ax) * M + q] + 0.5 * d * d * J[(size_t)(4 + ax) * M + q];
        acc -= s * jv / p.h2;
    }
    G[p.irr_node[r]] += acc;
}

template <int C>
__global__ __launch_bounds__(256) void k_rows3(DevPlan3 p, double* __restrict__ G, const int* __restrict__ skip) {
    if (skip && *skip) return;
    const int lane = threadIdx.x & 63;
    const int n = p.N - 1;
    const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= n * n) return;
    const int kk = r / n, jj = r % n;
    double* row = G + ((size_t)kk * p.N + jj) * p.N;
    double e[C];
#pragma unroll
    for (int c = 0; c < C; ++c) e[c] = row[lane * C + c] * p.h2;
    mode_solve<C>(e, p.modes[r], lane, p.N);
#pragma unroll
    for (int c = 0; c < C; ++c) row[lane * C + c] = e[c];
}

__device__ __forceinline__ double interp3_at(const DevPlan3& p, const double* __restrict__ G,
                                             const double* __restrict__ J, int m) {
    const int M = p.M;
    double v = 0.0;
#pragma unroll
    for (int s = 0; s < kStencil3; ++s) {
        const int node = p.st_node[(size_t)kStencil3 * m + s];
        const double gv = node >= 0 ? G[node] : 0.0;
        v = fma(p.st_w[(size_t)kStencil3 * m + s], gv, v);
    }
#pragma unroll
    for (int c = 0; c < kJump3; ++c) v = fma(p.st_t[(size_t)kJump3 * m + c], J[(size_t)c * M + m], v);
    return v;
}

__global__ __launch_bounds__(256) void k_interp3(DevPlan3 p, const double* __restrict__ G,
                                                 const double* __restrict__ J, double* __restrict__ out) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m < p.M) out[m] = interp3_at(p, G, J, m);
}

// inside GMRES: v+ at 64 control points, then the first Gram-Schmidt pass
__global__ __launch_bounds__(1024) void k_interp3_gm(DevPlan3 p, const double* __restrict__ G,
                                                     const double* __restrict__ J, GmresBufs b) {
    __shared__ double red[64];
    if (b.st->converged) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m = blockIdx.x * 64 + lane;
    if (wave == 0) {
        const double v = m < p.M ? interp3_at(p, G, J, m) : 0.0;
        if (m < p.M) b.w[m] = v;
        red[lane] = v;
    }
    __syncthreads();
    gm_dots1_64(b, p.M, blockIdx.x, red);
}

__global__ __launch_bounds__(256) void k_grid_out3(DevPlan3 p, const double* __restrict__ G, int mask,
                                                   double* __restrict__ u) {
    const int N = p.N, W = N + 1;
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)W * W * W) return;
    const int i = (int)(idx % W), j = (int)((idx / W) % W), k = (int)(idx / ((size_t)W * W));
    double v = 0.0;
    if (i >= 1 && j >= 1 && k >= 1 && i < N && j < N && k < N) v = G[((size_t)(k - 1) * N + (j - 1)) * N + (i - 1)];
    if (mask && !p.inside[idx]) v = 0.0;
    u[idx] = v;
}

}  // namespace

hipError_t launch_jumps3(const DevPlan3& p, const double* phi, const double* fgam, double* J, const int* skip,
                         hipStream_t s) {
    const size_t threads = (size_t)p.M * kFitLanes;
    if (hipError_t e = klaunch(&k_jumps3, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, p, phi, fgam, J,
                               skip))
        return e;
    return hipGetLastError();
}

hipError_t launch_fill3(const DevPlan3& p, const double* f, double* G, const int* skip, hipStream_t s) {
    const size_t tot = (size_t)p.N * p.N * p.N;
    if (hipError_t e = klaunch(&k_fill3, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, p, f, G, skip))
        return e;
    return hipGetLastError();
}

hipError_t launch_correct3(const DevPlan3& p, const double* J, double* G, const int* skip, hipStream_t s) {
    if (p.I == 0) return hipSuccess;
    if (hipError_t e = klaunch(&k_correct3, dim3((p.I + 255) / 256), dim3(256), 0, s, p, J, G, skip)) return e;
    return hipGetLastError();
}

hipError_t launch_solve3(const DevPlan3& p, double* G, int B, const int* skip, hipStream_t s) {
    const int N = p.N;
    const size_t plane = (size_t)N * N;
    const double inv = 2.0 / N;
    // along z: N^2 columns of N rows, rows N^2 apart
    if (hipError_t e = launch_dst_lines(N, p.log2N, p.sinq, G, 1.0, B, N * N, 1, 0, skip, s)) return e;
    // along y: each of the N-1 interior planes, rows N apart
    if (hipError_t e = launch_dst_lines(N, p.log2N, p.sinq, G, 1.0, B, N, N - 1, plane, skip, s)) return e;
    const int rows = (N - 1) * (N - 1);
    const dim3 g((rows + 3) / 4), t(256);
    hipError_t e = hipSuccess;
    switch (N) {
        case 64: e = klaunch(&k_rows3<1>, g, t, 0, s, p, G, skip); break;
        case 128: e = klaunch(&k_rows3<2>, g, t, 0, s, p, G, skip); break;
        case 256: e = klaunch(&k_rows3<4>, g, t, 0, s, p, G, skip); break;
        default: return hipErrorInvalidValue;
    }
    if (e) return e;
    if (hipError_t e2 = launch_dst_lines(N, p.log2N, p.sinq, G, inv, B, N, N - 1, plane, skip, s)) return e2;
    return launch_dst_lines(N, p.log2N, p.sinq, G, inv, B, N * N, 1, 0, skip, s);
}

hipError_t launch_interp3(const DevPlan3& p, const double* G, const double* J, double* out, const GmresBufs* gm,
                          hipStream_t s) {
    if (gm) return klaunch(&k_interp3_gm, dim3((p.M + 63) / 64), dim3(1024), 0, s, p, G, J, *gm);
    if (hipError_t e = klaunch(&k_interp3, dim3((p.M + 255) / 256), dim3(256), 0, s, p, G, J, out)) return e;
    return hipGetLastError();
}

hipError_t launch_grid_out3(const DevPlan3& p, const double* G, bool mask, double* u, hipStream_t s) {
    const size_t tot = (size_t)(p.N + 1) * (p.N + 1) * (p.N + 1);
    if (hipError_t e = klaunch(&k_grid_out3, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, p, G,
                               mask ? 1 : 0, u))
        return e;
    return hipGetLastError();
}

}  // namespace kfbi
