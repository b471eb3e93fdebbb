// HIP kernels of the KFBI hot path for gfx950 (MI355X), FP64.
//
// One K_D apply (Sec. 3, Alg. 1 steps 4-6) is three launches:
//   k_correct  one thread per irregular node: jumps at the crossings on its
//              arms (Alg. 2 line 4) and the correction of its right-hand side
//              (Alg. 2 line 5).  For the double-layer apply F = 0, so the
//              right-hand side of the corrected system is nonzero only here.
//   k_modes    the fast solver (Alg. 4) restricted to what the interpolation
//              reads.  Along y the right-hand side is expanded in sines; for a
//              sparse right-hand side each coefficient is a short sum over the
//              irregular nodes of one grid column.  Along x each sine mode is a
//              constant-coefficient tridiagonal system, solved by one wavefront
//              as two first-order recurrences (chunked, with wave-wide carry
//              scans) plus a rank-one boundary fix.  The inverse sine sum along
//              y is evaluated only at the six stencil nodes of each boundary
//              sample, already weighted by the interpolation weights, and summed
//              per workgroup into a partial result.
//   k_interp   one thread per sample: the partials summed in a fixed order plus
//              the jump terms of the stencil nodes outside Omega (Alg. 3).
// The dense solve (volume potential, final solution) uses the same tridiagonal
// solver on full rows, with the sine expansions along y done as products with
// the sine matrix (k_sine_gemm).
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace kfbi {

namespace {

// sin(pi m / N), 0 <= m < 2N, from the quarter-period table sq[0..N/2].
__device__ __forceinline__ double sinpi_n(const double* __restrict__ sq, int m, int N) {
    const double sgn = (m & N) ? -1.0 : 1.0;
    m &= N - 1;
    m = min(m, N - m);
    return sgn * sq[m];
}

// Second derivative of the periodic spline through y at sample m: the inverse
// of the (1, 4, 1) circulant decays like (2 - sqrt 3)^|k|, so a filter of
// 2K+3 taps reproduces it to double precision.
__device__ double spline_s2(const double* __restrict__ y, int M, const double* __restrict__ taps, int K, int m) {
    double s = 0.0;
    for (int q = -K - 1; q <= K + 1; ++q) {
        int idx = (m + q) % M;
        if (idx < 0) idx += M;
        s += taps[q + K + 1] * y[idx];
    }
    return s;
}

__device__ void spline_at(const double* __restrict__ y, const DevPlan& p, int seg, double u, double& v,
                          double& d1, double& d2) {
    const int k1 = seg + 1 == p.M ? 0 : seg + 1;
    const double s0 = spline_s2(y, p.M, p.taps, p.K, seg);
    const double s1 = spline_s2(y, p.M, p.taps, p.K, k1);
    const double y0 = y[seg], y1 = y[k1], w = 1.0 - u;
    const double sixth = 1.0 / 6.0;
    v = w * y0 + u * y1 + (w * w * w - w) * s0 * sixth + (u * u * u - u) * s1 * sixth;
    d1 = (y1 - y0) - (3.0 * w * w - 1.0) * s0 * sixth + (3.0 * u * u - 1.0) * s1 * sixth;
    d2 = w * s0 + u * s1;
}

struct J6 {
    double v, gx, gy, hxx, hxy, hyy;
};

// Cartesian jumps of the interface problem at one point of Gamma.
// [v] = Phi and [d_n v] = 0 (Sec. 2.2); differentiating along arc length gives
// [v_tau] = Phi_s, [v_tautau] = Phi_ss, [v_taun] = -c Phi_s; the equation gives
// [v_nn] = [F] + kappa Phi - [v_tautau].
__device__ J6 jumps_at(const DevPlan& p, const PointGeom& g, const double* __restrict__ phi,
                       const double* __restrict__ fgam) {
    double P = 0.0, P1 = 0.0, P2 = 0.0, F = 0.0, t1, t2;
    if (phi) spline_at(phi, p, g.seg, g.u, P, P1, P2);
    if (fgam) spline_at(fgam, p, g.seg, g.u, F, t1, t2);
    const double Ps = P1 * g.a1;
    const double Pss = P2 * g.a2 - P1 * g.a3;
    const double vtt = Pss, vtn = -g.curv * Ps, vnn = F + p.kappa * P - vtt;
    J6 J;
    J.v = P;
    J.gx = Ps * g.tx;
    J.gy = Ps * g.ty;
    J.hxx = vtt * g.tx * g.tx + 2.0 * vtn * g.tx * g.nx + vnn * g.nx * g.nx;
    J.hxy = vtt * g.tx * g.ty + vtn * (g.tx * g.ny + g.nx * g.ty) + vnn * g.nx * g.ny;
    J.hyy = vtt * g.ty * g.ty + 2.0 * vtn * g.ty * g.ny + vnn * g.ny * g.ny;
    return J;
}

// ---------------------------------------------------------------- correction (Alg. 2)

__global__ __launch_bounds__(256) void k_correct(DevPlan p, JumpSrc js, double* __restrict__ corr,
                                                 double* __restrict__ dense, const int* __restrict__ skip) {
    if (skip && *skip) return;
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= p.I) return;
    const double s = p.irr_s[r];
    double acc = 0.0;
    for (int a = 0; a < 4; ++a) {
        const int k = p.arm_q[4 * r + a];
        if (k < 0) break;
        const double d = p.arm_d[4 * r + a];
        const int ax = p.q_axis[k];
        double v, g, hh;
        if (js.jq) {
            const double* J = js.jq + 6 * (size_t)k;
            v = J[0];
            g = ax ? J[2] : J[1];
            hh = ax ? J[5] : J[3];
        } else {
            const J6 J = jumps_at(p, p.q_geo[k], js.phi, js.fgam);
            v = J.v;
            g = ax ? J.gy : J.gx;
            hh = ax ? J.hyy : J.hxx;
        }
        // jump continued along the arm to the neighbour across Gamma
        acc -= s * (v + d * g + 0.5 * d * d * hh);
    }
    acc *= p.inv_h2;
    if (corr) corr[r] = acc;
    if (dense) dense[(size_t)(p.irr_j[r] - 1) * p.N + (p.irr_i[r] - 1)] += acc;
}

// ---------------------------------------------------------------- tridiagonal mode solve (Alg. 4)
//
// Solve x[i-1] - beta x[i] + x[i+1] = e[i], i = 1..N-1, x[0] = x[N] = 0, with
// tridiag(1, -beta, 1) = -(1/r)(I - r S)(I - r S^T) - r e1 e1^T (S the down
// shift): the forward recurrence w[i] = r (w[i-1] - e[i]), the backward one
// y[i] = w[i] + r y[i+1], and x = y + y[1] zeta with
// zeta[i] = -r (r^i - r^(2N-i)) / (1 - r^(2N)) from the rank-one term.
// Lane L of the wavefront owns i = L C + 1 .. L C + C (i = N is a zero pad);
// each recurrence runs locally per lane and the lanes are joined by a scan of
// the carries with multiplier r^C.
template <int C>
__device__ __forceinline__ void mode_solve(double (&e)[C], const ModeConst& mc, int lane, int N) {
    const double r = mc.r;
    double w = 0.0;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        w = r * (w - e[c]);
        e[c] = w;
    }
    double val = w, mul = mc.rC;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const double t = __shfl_up(val, off, 64);
        if (lane >= off) val += mul * t;
        mul *= mul;
    }
    double carry = __shfl_up(val, 1, 64);
    if (lane == 0) carry = 0.0;
    double pw = r;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        e[c] += pw * carry;
        pw *= r;
    }
    if (lane == 63) e[C - 1] = 0.0;
    double y = 0.0;
#pragma unroll
    for (int c = C - 1; c >= 0; --c) {
        y = e[c] + r * y;
        e[c] = y;
    }
    val = y;
    mul = mc.rC;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const double t = __shfl_down(val, off, 64);
        if (lane + off < 64) val += mul * t;
        mul *= mul;
    }
    carry = __shfl_down(val, 1, 64);
    if (lane == 63) carry = 0.0;
    pw = r;
#pragma unroll
    for (int c = C - 1; c >= 0; --c) {
        e[c] += pw * carry;
        pw *= r;
    }
    const double y1 = __shfl(e[0], 0, 64);
    const int is = lane * C + 1;
    double p1 = exp((double)is * mc.logr);
    double p2 = exp((double)(2 * N - is) * mc.logr);
    const double coef = y1 * mc.smc;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        e[c] += coef * (p1 - p2);
        p1 *= r;
        p2 *= mc.rinv;
    }
    if (lane == 63) e[C - 1] = 0.0;
}

// ---------------------------------------------------------------- sparse fast solve + weighted gather

template <int C, int W>
__global__ __launch_bounds__(W * 64) void k_modes(DevPlan p, const double* __restrict__ corr,
                                                  double* __restrict__ partial, const int* __restrict__ skip) {
    if (skip && *skip) return;
    extern __shared__ double smem[];
    const int N = p.N, n = p.n, M = p.M, mask2 = 2 * N - 1;
    double* sq = smem;                       // N/2 + 2
    double* xs = sq + (N / 2 + 2);           // W (N + 1)
    double* acc = xs + W * (N + 1);          // M
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int k = tid; k <= N / 2; k += W * 64) sq[k] = p.sinq[k];
    for (int k = tid; k < M; k += W * 64) acc[k] = 0.0;
    __syncthreads();
    for (int base = blockIdx.x * W; base < n; base += gridDim.x * W) {
        const int l = base + wave + 1;
        double* x = xs + wave * (N + 1);
        if (l <= n) {
            double e[C];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const int i = lane * C + 1 + c;
                double s = 0.0;
                if (i <= n) {
                    const int b = p.col_ptr[i], en = p.col_ptr[i + 1];
                    for (int q = b; q < en; ++q) s += corr[q] * sinpi_n(sq, (p.irr_j[q] * l) & mask2, N);
                }
                e[c] = s * p.h2;
            }
            mode_solve<C>(e, p.modes[l], lane, N);
            if (lane == 0) x[0] = 0.0;
#pragma unroll
            for (int c = 0; c < C; ++c) x[lane * C + 1 + c] = e[c];
        }
        __syncthreads();
        for (int cp = tid; cp < M; cp += W * 64) {
            const int i0 = p.cp_i0[cp], j0 = p.cp_j0[cp], sxy = p.cp_sxy[cp];
            const int sx = (sxy & 1) ? 1 : -1;
            const bool syp = (sxy & 2) != 0;
            const double* w = p.cp_w + 6 * (size_t)cp;
            const double w0 = w[0], wE = w[1], wW = w[2], wN = w[3], wS = w[4], wD = w[5];
            double s = 0.0;
            for (int q = 0; q < W; ++q) {
                const int lq = base + q + 1;
                if (lq > n) break;
                const double* xq = xs + q * (N + 1);
                const double s0 = sinpi_n(sq, (j0 * lq) & mask2, N);
                const double sp = sinpi_n(sq, ((j0 + 1) * lq) & mask2, N);
                const double sm = sinpi_n(sq, ((j0 - 1) * lq) & mask2, N);
                const double xc = xq[i0];
                s += s0 * (w0 * xc + wE * xq[i0 + 1] + wW * xq[i0 - 1]) + sp * wN * xc + sm * wS * xc +
                     (syp ? sp : sm) * wD * xq[i0 + sx];
            }
            acc[cp] += s;
        }
        __syncthreads();
    }
    for (int cp = tid; cp < M; cp += W * 64) partial[(size_t)blockIdx.x * M + cp] = acc[cp];
}

// ---------------------------------------------------------------- interpolation (Alg. 3)

__global__ __launch_bounds__(256) void k_interp(DevPlan p, JumpSrc js, const double* __restrict__ partial, int G,
                                                const double* __restrict__ R, double* __restrict__ out,
                                                const int* __restrict__ skip) {
    if (skip && *skip) return;
    const int cp = blockIdx.x * blockDim.x + threadIdx.x;
    if (cp >= p.M) return;
    const int i0 = p.cp_i0[cp], j0 = p.cp_j0[cp], sxy = p.cp_sxy[cp];
    const int sx = (sxy & 1) ? 1 : -1, sy = (sxy & 2) ? 1 : -1;
    const int ni[6] = {i0, i0 + 1, i0 - 1, i0, i0, i0 + sx};
    const int nj[6] = {j0, j0, j0, j0 + 1, j0 - 1, j0 + sy};
    const double* w = p.cp_w + 6 * (size_t)cp;
    double s = 0.0;
    if (partial) {
        for (int g = 0; g < G; ++g) s += partial[(size_t)g * p.M + cp];
        s *= 2.0 / p.N;
    } else {
        for (int k = 0; k < 6; ++k) s += w[k] * R[(size_t)(nj[k] - 1) * p.N + (ni[k] - 1)];
    }
    const unsigned char* o6 = p.cp_out + 6 * (size_t)cp;
    const bool any = o6[0] | o6[1] | o6[2] | o6[3] | o6[4] | o6[5];
    if (any) {
        J6 J;
        if (js.jz) {
            const double* q = js.jz + 6 * (size_t)cp;
            J = {q[0], q[1], q[2], q[3], q[4], q[5]};
        } else {
            J = jumps_at(p, p.z_geo[cp], js.phi, js.fgam);
        }
        const double zx = p.zx[cp], zy = p.zy[cp];
        for (int k = 0; k < 6; ++k) {
            if (!o6[k]) continue;
            const double dx = p.lo + ni[k] * p.h - zx, dy = p.lo + nj[k] * p.h - zy;
            s += w[k] * (J.v + dx * J.gx + dy * J.gy + 0.5 * (dx * dx * J.hxx + 2.0 * dx * dy * J.hxy + dy * dy * J.hyy));
        }
    }
    out[cp] = s;
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

// C = alpha S B with S[l][j] = sin(pi (l+1)(j+1) / N): the sine expansion along
// y of every column at once (both the forward and the inverse transform).
// 64 x 64 output tile per workgroup, 4 x 4 outputs per thread, k-tiles of 16.
__global__ __launch_bounds__(256) void k_sine_gemm(int N, const double* __restrict__ sinq,
                                                   const double* __restrict__ B, double* __restrict__ Cm,
                                                   double alpha) {
    __shared__ double sq[2050];
    __shared__ double As[16][65];
    __shared__ double Bs[16][64];
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    const int row0 = blockIdx.y * 64, col0 = blockIdx.x * 64;
    const int mask2 = 2 * N - 1;
    for (int k = tid; k <= N / 2; k += 256) sq[k] = sinq[k];
    __syncthreads();
    double c[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) c[a][b] = 0.0;
    for (int k0 = 0; k0 < N; k0 += 16) {
        for (int t = tid; t < 1024; t += 256) {
            const int rr = t & 63, kk = t >> 6;
            As[kk][rr] = sinpi_n(sq, ((row0 + rr + 1) * (k0 + kk + 1)) & mask2, N);
            const int kb = t >> 6, cc = t & 63;
            Bs[kb][cc] = B[(size_t)(k0 + kb) * N + col0 + cc];
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            double a[4], b[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                a[q] = As[kk][ty + 16 * q];
                b[q] = Bs[kk][tx + 16 * q];
            }
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int r = 0; r < 4; ++r) c[q][r] = fma(a[q], b[r], c[q][r]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) Cm[(size_t)(row0 + ty + 16 * q) * N + col0 + tx + 16 * r] = alpha * c[q][r];
}

// One wavefront per sine mode l (row l-1 of A): the tridiagonal solve along x.
template <int C>
__global__ __launch_bounds__(256) void k_rows_solve(DevPlan p, double* __restrict__ A) {
    const int lane = threadIdx.x & 63;
    const int l = blockIdx.x * 4 + (threadIdx.x >> 6) + 1;
    if (l > p.n) return;
    double* row = A + (size_t)(l - 1) * p.N;
    double e[C];
#pragma unroll
    for (int c = 0; c < C; ++c) e[c] = row[lane * C + c] * p.h2;
    mode_solve<C>(e, p.modes[l], lane, p.N);
#pragma unroll
    for (int c = 0; c < C; ++c) row[lane * C + c] = e[c];
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

// ---------------------------------------------------------------- GMRES step (Alg. 5)

__device__ double block_sum(double v, double* red) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
    for (int k = 0; k < nw; ++k) s += red[k];
    return s;
}

// One step of restarted GMRES, driven by a state machine in device memory so
// that the host only polls for convergence.  Mode 0: b.w holds K_D phi; form
// the true residual, stop or start a cycle.  Mode 1: b.w holds K_D V_j;
// orthogonalise it (classical Gram-Schmidt applied twice), extend the
// Hessenberg matrix, update the Givens rotations and the residual estimate;
// at the end of a cycle solve the small triangular system and update phi.
__global__ __launch_bounds__(1024) void k_gmres(GmresBufs b, int M) {
    __shared__ double red[16];
    __shared__ double hs[128];
    __shared__ double ys[128];
    __shared__ int s_end;
    GmresState* st = b.st;
    if (st->converged) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m = b.m, mode = st->mode, j = st->j, it = st->it, first = st->first;
    const double r0_in = st->r0;
    __syncthreads();
    if (mode == 0) {
        double part = 0.0;
        for (int e = tid; e < M; e += 1024) {
            const double r = b.ghat[e] - b.w[e];
            b.V[e] = r;
            part += r * r;
        }
        const double beta = sqrt(block_sum(part, red));
        const double r0 = first ? beta : r0_in;
        const double rel = r0 > 0.0 ? beta / r0 : 0.0;
        const bool done = r0 == 0.0 || beta == 0.0 || rel < b.tol || it >= b.max_iter;
        if (!done) {
            const double ib = 1.0 / beta;
            for (int e = tid; e < M; e += 1024) {
                const double v = b.V[e] * ib;
                b.V[e] = v;
                b.xcur[e] = v;
            }
        }
        if (tid == 0) {
            st->r0 = r0;
            st->first = 0;
            st->relres = rel;
            if (done) {
                st->converged = (r0 == 0.0 || beta == 0.0 || rel < b.tol) ? 1 : -1;
                st->mode = 2;
            } else {
                b.g[0] = beta;
                for (int k = 1; k <= m; ++k) b.g[k] = 0.0;
                st->j = 0;
                st->mode = 1;
                st->cycles += 1;
            }
        }
        return;
    }
    // mode 1: Arnoldi column j
    double* Hj = b.H + (size_t)j * (m + 1);
    for (int pass = 0; pass < 2; ++pass) {
        for (int i = wave; i <= j; i += 16) {
            const double* Vi = b.V + (size_t)i * M;
            double d = 0.0;
            for (int e = lane; e < M; e += 64) d += Vi[e] * b.w[e];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) d += __shfl_xor(d, off, 64);
            if (lane == 0) hs[i] = d;
        }
        __syncthreads();
        for (int e = tid; e < M; e += 1024) {
            double a = b.w[e];
            for (int i = 0; i <= j; ++i) a -= hs[i] * b.V[(size_t)i * M + e];
            b.w[e] = a;
        }
        if (tid <= j) Hj[tid] = (pass == 0 ? 0.0 : Hj[tid]) + hs[tid];
        __syncthreads();
    }
    double part = 0.0;
    for (int e = tid; e < M; e += 1024) part += b.w[e] * b.w[e];
    const double hn = sqrt(block_sum(part, red));
    const double ihn = hn > 0.0 ? 1.0 / hn : 0.0;
    double* Vn = b.V + (size_t)(j + 1) * M;
    for (int e = tid; e < M; e += 1024) Vn[e] = b.w[e] * ihn;
    if (tid == 0) {
        for (int i = 0; i < j; ++i) {
            const double a = Hj[i], c = Hj[i + 1];
            Hj[i] = b.cs[i] * a + b.sn[i] * c;
            Hj[i + 1] = -b.sn[i] * a + b.cs[i] * c;
        }
        const double den = hypot(Hj[j], hn);
        const double cs = den > 0.0 ? Hj[j] / den : 1.0;
        const double sn = den > 0.0 ? hn / den : 0.0;
        b.cs[j] = cs;
        b.sn[j] = sn;
        Hj[j] = den;
        Hj[j + 1] = 0.0;
        const double gj = b.g[j];
        b.g[j + 1] = -sn * gj;
        b.g[j] = cs * gj;
        const int jn = j + 1, itn = it + 1;
        const double est = fabs(b.g[jn]) / r0_in;
        st->relres = est;
        st->it = itn;
        const bool end = est < b.tol || jn == m || itn >= b.max_iter || hn == 0.0;
        s_end = end ? 1 : 0;
        if (end) {
            // back substitution H[0:jn, 0:jn] y = g[0:jn]
            for (int i = jn - 1; i >= 0; --i) {
                double a = b.g[i];
                for (int k = i + 1; k < jn; ++k) a -= b.H[(size_t)k * (m + 1) + i] * ys[k];
                ys[i] = a / b.H[(size_t)i * (m + 1) + i];
            }
            st->mode = 0;
        } else {
            st->j = jn;
        }
    }
    __syncthreads();
    if (s_end) {
        const int jn = j + 1;
        for (int e = tid; e < M; e += 1024) {
            double a = b.phi[e];
            for (int i = 0; i < jn; ++i) a += ys[i] * b.V[(size_t)i * M + e];
            b.phi[e] = a;
            b.xcur[e] = a;
        }
    } else {
        for (int e = tid; e < M; e += 1024) b.xcur[e] = Vn[e];
    }
}

template <int C>
hipError_t modes_dispatch_w(const DevPlan& p, const double* corr, double* partial, int G, int W, const int* skip,
                            hipStream_t s) {
    const size_t lds = modes_lds_bytes(p.N, p.M, W);
    switch (W) {
        case 4:
            hipFuncSetAttribute((const void*)k_modes<C, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            k_modes<C, 4><<<G, 256, lds, s>>>(p, corr, partial, skip);
            break;
        case 2:
            hipFuncSetAttribute((const void*)k_modes<C, 2>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            k_modes<C, 2><<<G, 128, lds, s>>>(p, corr, partial, skip);
            break;
        default:
            hipFuncSetAttribute((const void*)k_modes<C, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            k_modes<C, 1><<<G, 64, lds, s>>>(p, corr, partial, skip);
            break;
    }
    return hipGetLastError();
}

template <int C>
hipError_t rows_dispatch(const DevPlan& p, double* A, hipStream_t s) {
    k_rows_solve<C><<<(p.n + 3) / 4, 256, 0, s>>>(p, A);
    return hipGetLastError();
}

}  // namespace

size_t modes_lds_bytes(int N, int M, int W) {
    return sizeof(double) * ((size_t)(N / 2 + 2) + (size_t)W * (N + 1) + (size_t)M);
}

hipError_t launch_correct(const DevPlan& p, JumpSrc js, double* corr, double* dense, const int* skip,
                          hipStream_t s) {
    if (p.I == 0) return hipSuccess;
    k_correct<<<(p.I + 255) / 256, 256, 0, s>>>(p, js, corr, dense, skip);
    return hipGetLastError();
}

hipError_t launch_modes(const DevPlan& p, const double* corr, double* partial, int G, int W, const int* skip,
                        hipStream_t s) {
    switch (p.N) {
        case 64: return modes_dispatch_w<1>(p, corr, partial, G, W, skip, s);
        case 128: return modes_dispatch_w<2>(p, corr, partial, G, W, skip, s);
        case 256: return modes_dispatch_w<4>(p, corr, partial, G, W, skip, s);
        case 512: return modes_dispatch_w<8>(p, corr, partial, G, W, skip, s);
        case 1024: return modes_dispatch_w<16>(p, corr, partial, G, W, skip, s);
        case 2048: return modes_dispatch_w<32>(p, corr, partial, G, W, skip, s);
        case 4096: return modes_dispatch_w<64>(p, corr, partial, G, W, skip, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_interp(const DevPlan& p, JumpSrc js, const double* partial, int G, const double* R, double* out,
                         const int* skip, hipStream_t s) {
    k_interp<<<(p.M + 255) / 256, 256, 0, s>>>(p, js, partial, G, R, out, skip);
    return hipGetLastError();
}

hipError_t launch_fill_rhs(const DevPlan& p, const double* f, bool mask, double* R, hipStream_t s) {
    const size_t tot = (size_t)p.N * p.N;
    k_fill_rhs<<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(p, f, mask ? 1 : 0, R);
    return hipGetLastError();
}

hipError_t launch_sine_gemm(const DevPlan& p, const double* B, double* Cm, double alpha, hipStream_t s) {
    if (p.N % 64 || p.N > 4096) return hipErrorInvalidValue;
    dim3 grid(p.N / 64, p.N / 64);
    k_sine_gemm<<<grid, 256, 0, s>>>(p.N, p.sinq, B, Cm, alpha);
    return hipGetLastError();
}

hipError_t launch_rows_solve(const DevPlan& p, double* A, hipStream_t s) {
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

hipError_t launch_grid_out(const DevPlan& p, const double* R, bool mask, double* u, hipStream_t s) {
    const size_t tot = (size_t)(p.N + 1) * (p.N + 1);
    k_grid_out<<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(p, R, mask ? 1 : 0, u);
    return hipGetLastError();
}

hipError_t launch_axpby(int n, double a, const double* x, double b, const double* y, double* z, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_axpby<<<(n + 255) / 256, 256, 0, s>>>(n, a, x, b, y, z);
    return hipGetLastError();
}

hipError_t launch_gmres_step(const DevPlan& p, GmresBufs b, hipStream_t s) {
    k_gmres<<<1, 1024, 0, s>>>(b, p.M);
    return hipGetLastError();
}

}  // namespace kfbi
