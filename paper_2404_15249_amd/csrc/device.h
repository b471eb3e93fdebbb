// Device functions shared by the single-problem and the batched kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.h"

namespace kfbi {

// A flag or state word another launch wrote, read through the vector memory
// path: such loads are waited for only where the value is used, where a scalar
// load here is waited for at once, before the loads issued after it.
__device__ __forceinline__ int load_flag(const int* f) {
    // a global (not flat) load: a flat load also counts as a scalar-memory
    // access, so the next wait for the kernel's arguments would wait for it too
    using global_int = __attribute__((address_space(1))) int;
    return __hip_atomic_load((global_int*)f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// load_flag for a value used only late in the kernel: the address is offset by
// a zero the compiler cannot see through, so the value stays per lane and is
// not moved to a scalar register (which waits for it) right after the load.
__device__ __forceinline__ int load_flag_late(const int* f) {
    int zero;
    asm volatile("v_mov_b32 %0, 0" : "=v"(zero));
    return load_flag(f + zero);
}
// A flag that is never set, read in place of a null one (a load from one of two
// addresses, with no branch that would wait for it).
static __device__ const int kFlagZero = 0;
__device__ __forceinline__ int load_flag_or_zero(const int* f) { return load_flag(f ? f : &kFlagZero); }


// sin(pi m / N), 0 <= m < 2N, from the quarter-period table sq[0..N/2].
__device__ __forceinline__ double sinpi_n(const double* __restrict__ sq, int m, int N) {
    const double sgn = (m & N) ? -1.0 : 1.0;
    m &= N - 1;
    m = min(m, N - m);
    return sgn * sq[m];
}

// Second derivative of the periodic spline through y at sample m: the inverse
// of the (1, 4, 1) circulant decays like (2 - sqrt 3)^|k|, so a filter of
// 2K+3 taps reproduces it to double precision.  Computed once per density by
// k_spline; the kernels below read the result.
__device__ inline double spline_s2(const double* __restrict__ y, int M, const double* __restrict__ taps, int m) {
    constexpr int K = kSplineK;
    double s = 0.0;
    if (M > K + 1 && m >= K + 1 && m + K + 1 < M) {
#pragma unroll
        for (int q = -K - 1; q <= K + 1; ++q) s = fma(taps[q + K + 1], y[m + q], s);
    } else {
#pragma unroll
        for (int q = -K - 1; q <= K + 1; ++q) {
            int idx = (m + q) % M;
            if (idx < 0) idx += M;
            s = fma(taps[q + K + 1], y[idx], s);
        }
    }
    return s;
}

// Value and first two parameter derivatives of the spline on segment seg at u.
__device__ __forceinline__ void spline_at(const double* __restrict__ y, const double* __restrict__ s2,
                                          const DevPlan& p, int seg, double u, double& v, double& d1, double& d2) {
    const int k1 = seg + 1 == p.M ? 0 : seg + 1;
    const double s0 = s2[seg], s1 = s2[k1];
    const double y0 = y[seg], y1 = y[k1], w = 1.0 - u;
    const double sixth = 1.0 / 6.0;
    v = w * y0 + u * y1 + (w * w * w - w) * s0 * sixth + (u * u * u - u) * s1 * sixth;
    d1 = (y1 - y0) - (3.0 * w * w - 1.0) * s0 * sixth + (3.0 * u * u - 1.0) * s1 * sixth;
    d2 = w * s0 + u * s1;
}

struct J6 {
    double v, gx, gy, hxx, hxy, hyy;
};

// Cartesian jumps of the interface problem at one point of Gamma.  With n the
// outward normal, c the curvature and the density D along arc length:
//   [v] = D, [d_n v] = 0 (Sec. 2.2):  [v_tau] = D_s, [v_tautau] = D_ss, [v_taun] = -c D_s;
//   [v] = 0, [d_n v] = D (Neumann):   [v_n] = D, [v_tautau] = c D, [v_taun] = D_s;
// and the equation gives [v_nn] = [F] + kappa [v] - [v_tautau].
// P, P1, P2: the density's spline value and parameter derivatives at the
// point; F: the jump of f there.
__device__ inline J6 jumps_from(const DevPlan& p, const PointGeom& g, double P, double P1, double P2, double F) {
    const double Ps = P1 * g.a1;
    J6 J;
    if (p.normal_jump) {
        const double vtt = g.curv * P, vtn = Ps, vnn = F - vtt;
        J.v = 0.0;
        J.gx = P * g.nx;
        J.gy = P * g.ny;
        J.hxx = vtt * g.tx * g.tx + 2.0 * vtn * g.tx * g.nx + vnn * g.nx * g.nx;
        J.hxy = vtt * g.tx * g.ty + vtn * (g.tx * g.ny + g.nx * g.ty) + vnn * g.nx * g.ny;
        J.hyy = vtt * g.ty * g.ty + 2.0 * vtn * g.ty * g.ny + vnn * g.ny * g.ny;
        return J;
    }
    const double Pss = P2 * g.a2 - P1 * g.a3;
    const double vtt = Pss, vtn = -g.curv * Ps, vnn = F + p.kappa * P - vtt;
    J.v = P;
    J.gx = Ps * g.tx;
    J.gy = Ps * g.ty;
    J.hxx = vtt * g.tx * g.tx + 2.0 * vtn * g.tx * g.nx + vnn * g.nx * g.nx;
    J.hxy = vtt * g.tx * g.ty + vtn * (g.tx * g.ny + g.nx * g.ty) + vnn * g.nx * g.ny;
    J.hyy = vtt * g.ty * g.ty + 2.0 * vtn * g.ty * g.ny + vnn * g.ny * g.ny;
    return J;
}

// The same at the point of segment g.seg, offset g.u, from the densities' splines.
__device__ inline J6 jumps_at(const DevPlan& p, const PointGeom& g, const JumpSrc& js) {
    double P = 0.0, P1 = 0.0, P2 = 0.0, F = 0.0, t1, t2;
    if (js.phi) spline_at(js.phi, js.phi_s2, p, g.seg, g.u, P, P1, P2);
    if (js.fgam) spline_at(js.fgam, js.fgam_s2, p, g.seg, g.u, F, t1, t2);
    return jumps_from(p, g, P, P1, P2, F);
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
// ---------------------------------------------------------------- wavefront scans with DPP
//
// A lane's FP64 value moved by a DPP control (row shifts stay inside rows of
// 16 lanes, wave shifts cross them); lanes without a source get 0.
constexpr int kDppRowShl1 = 0x101, kDppRowShr1 = 0x111, kDppWaveShl1 = 0x130, kDppWaveShr1 = 0x138;

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double readlane_f64(double v, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

// The sum over the wavefront, the same in every lane: the partner lane of each
// step differs in one more bit of the lane index (DPP quad swaps for bits 0
// and 1, the half-row and row mirrors, lane ^ 7 and lane ^ 15, for bits 2 and
// 3), so every lane holds its row's sum after four steps; the four row sums
// are then read as scalars.  Each step adds the same two values in either
// partner, so all lanes agree to the bit.
constexpr int kDppQuadSwap1 = 0xB1, kDppQuadSwap2 = 0x4E, kDppRowMirror = 0x140, kDppRowHalfMirror = 0x141;
__device__ __forceinline__ double wave_allsum(double v) {
    v += dpp_f64<kDppQuadSwap1>(v);
    v += dpp_f64<kDppQuadSwap2>(v);
    v += dpp_f64<kDppRowHalfMirror>(v);
    v += dpp_f64<kDppRowMirror>(v);
    return (readlane_f64(v, 0) + readlane_f64(v, 16)) + (readlane_f64(v, 32) + readlane_f64(v, 48));
}

// base^k for 0 <= k < 256 by repeated squaring (eight fixed steps)
__device__ __forceinline__ double pow_u8(double base, int k) {
    double res = 1.0;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        if ((k >> b) & 1) res *= base;
        base *= base;
    }
    return res;
}

// Weighted inclusive scans over the wavefront, v_L <- sum_k m^|L-k| v_k over
// k <= L (up) or k >= L (down): inside each row of 16 lanes by four DPP row
// shifts, then across the rows from the row ends read as scalars.
__device__ __forceinline__ double wave_scan_up(double v, double m, int lane) {
    const double m2 = m * m, m4 = m2 * m2, m8 = m4 * m4, m16 = m8 * m8;
    v = fma(m, dpp_f64<kDppRowShr1>(v), v);
    v = fma(m2, dpp_f64<kDppRowShr1 + 1>(v), v);
    v = fma(m4, dpp_f64<kDppRowShr1 + 3>(v), v);
    v = fma(m8, dpp_f64<kDppRowShr1 + 7>(v), v);
    const double p0 = readlane_f64(v, 15);
    const double p1 = fma(m16, p0, readlane_f64(v, 31));
    const double p2 = fma(m16, p1, readlane_f64(v, 47));
    const int row = lane >> 4;
    const double before = row == 0 ? 0.0 : row == 1 ? p0 : row == 2 ? p1 : p2;
    return fma(pow_u8(m, (lane & 15) + 1), before, v);
}

__device__ __forceinline__ double wave_scan_down(double v, double m, int lane) {
    const double m2 = m * m, m4 = m2 * m2, m8 = m4 * m4, m16 = m8 * m8;
    v = fma(m, dpp_f64<kDppRowShl1>(v), v);
    v = fma(m2, dpp_f64<kDppRowShl1 + 1>(v), v);
    v = fma(m4, dpp_f64<kDppRowShl1 + 3>(v), v);
    v = fma(m8, dpp_f64<kDppRowShl1 + 7>(v), v);
    const double q3 = readlane_f64(v, 48);
    const double q2 = fma(m16, q3, readlane_f64(v, 32));
    const double q1 = fma(m16, q2, readlane_f64(v, 16));
    const int row = lane >> 4;
    const double after = row == 3 ? 0.0 : row == 2 ? q3 : row == 1 ? q2 : q1;
    return fma(pow_u8(m, 16 - (lane & 15)), after, v);
}

template <int C>
__device__ __forceinline__ void mode_solve(double (&e)[C], const ModeConst& mc, int lane, int N) {
    const double r = mc.r, rinv = mc.rinv;
    // forward recurrence w = r (w - e): one dependent fma per step
    double w = 0.0;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const double re = r * e[c];
        w = fma(r, w, -re);
        e[c] = w;
    }
    // the lanes' carries: the weighted prefix of the chunk ends, from lane L-1
    double carry = dpp_f64<kDppWaveShr1>(wave_scan_up(w, mc.rC, lane));
    // e[c] += r^(c+1) carry; the powers in four interleaved chains
    const double r2 = r * r, r4 = r2 * r2;
    double pw[4] = {r, r2, r2 * r, r4};
#pragma unroll
    for (int c = 0; c < C; ++c) {
        e[c] = fma(pw[c & 3], carry, e[c]);
        pw[c & 3] *= r4;
    }
    if (lane == 63) e[C - 1] = 0.0;
    double y = 0.0;
#pragma unroll
    for (int c = C - 1; c >= 0; --c) {
        y = fma(r, y, e[c]);
        e[c] = y;
    }
    carry = dpp_f64<kDppWaveShl1>(wave_scan_down(y, mc.rC, lane));
    // e[c] += r^(C-c) carry
    pw[0] = r;
    pw[1] = r2;
    pw[2] = r2 * r;
    pw[3] = r4;
#pragma unroll
    for (int c = C - 1; c >= 0; --c) {
        const int k = (C - 1 - c) & 3;
        e[c] = fma(pw[k], carry, e[c]);
        pw[k] *= r4;
    }
    // rank-one fix: e[c] += y1 smc (r^i - r^(2N-i)) at i = lane C + 1 + c, with
    // r^(lane C + 1) = r (r^C)^lane and r^(2N - lane C - 1) = (r^C)^(128 - lane) / r
    // (2N = 128 C); the powers along c again in four chains
    const double y1 = readlane_f64(e[0], 0);
    const double coef = y1 * mc.smc;
    const double p1 = r * pow_u8(mc.rC, lane);
    const double p2 = rinv * pow_u8(mc.rC, 128 - lane);
    const double ri2 = rinv * rinv, ri4 = ri2 * ri2;
    double pa[4] = {p1, p1 * r, p1 * r2, p1 * r2 * r};
    double pb[4] = {p2, p2 * rinv, p2 * ri2, p2 * ri2 * rinv};
#pragma unroll
    for (int c = 0; c < C; ++c) {
        e[c] = fma(coef, pa[c & 3] - pb[c & 3], e[c]);
        pa[c & 3] *= r4;
        pb[c & 3] *= ri4;
    }
    if (lane == 63) e[C - 1] = 0.0;
}

// mode_solve on a wavefront's padded solution in LDS (node i at
// i + (i - 1) / C, values scaled by h2 on the way in), for chunks too long to
// keep in registers: the same steps, streamed through LDS.
template <int C>
__device__ __forceinline__ void mode_solve_lds(double* x, const ModeConst& mc, int lane, int N, double h2) {
    double* e = x + lane * (C + 1) + 1;
    const double r = mc.r;
    double w = 0.0;
#pragma unroll 8
    for (int c = 0; c < C; ++c) {
        w = r * (w - e[c] * h2);
        e[c] = w;
    }
    double carry = dpp_f64<kDppWaveShr1>(wave_scan_up(w, mc.rC, lane));
    double pw = r;
#pragma unroll 8
    for (int c = 0; c < C; ++c) {
        e[c] += pw * carry;
        pw *= r;
    }
    if (lane == 63) e[C - 1] = 0.0;
    double y = 0.0;
#pragma unroll 8
    for (int c = C - 1; c >= 0; --c) {
        y = e[c] + r * y;
        e[c] = y;
    }
    carry = dpp_f64<kDppWaveShl1>(wave_scan_down(y, mc.rC, lane));
    pw = r;
#pragma unroll 8
    for (int c = C - 1; c >= 0; --c) {
        e[c] += pw * carry;
        pw *= r;
    }
    const double y1 = readlane_f64(e[0], 0);
    double p1 = r * pow_u8(mc.rC, lane);                    // r^(lane C + 1)
    double p2 = mc.rinv * pow_u8(mc.rC, 128 - lane);        // r^(2N - lane C - 1), 2N = 128 C
    const double coef = y1 * mc.smc;
#pragma unroll 8
    for (int c = 0; c < C; ++c) {
        e[c] += coef * (p1 - p2);
        p1 *= r;
        p2 *= mc.rinv;
    }
    if (lane == 63) e[C - 1] = 0.0;
}

// Jump terms of the stencil nodes outside Omega: the far-side value is moved to
// the Omega side with the Taylor expansion of the jumps at the sample.  Every
// load is issued before any is used: sample cp is the knot that starts spline
// segment cp (u = 0, as the plan builds it), so the density's values there do
// not wait for the sample's geometry.
__device__ inline double outside_terms(const DevPlan& p, const JumpSrc& js, int cp, const int (&ni)[6], const int (&nj)[6],
                                const double* __restrict__ w) {
    const unsigned char* o6 = p.cp_out + 6 * (size_t)cp;
    unsigned char o[6];
    double wk[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        o[k] = o6[k];
        wk[k] = w[k];
    }
    const PointGeom g = p.z_geo[cp];
    const double zx = p.zx[cp], zy = p.zy[cp];
    J6 J;
    if (js.jz) {
        const double* q = js.jz + 6 * (size_t)cp;
        J = {q[0], q[1], q[2], q[3], q[4], q[5]};
    } else {
        double P = 0.0, P1 = 0.0, P2 = 0.0, F = 0.0, t1, t2;
        if (js.phi) spline_at(js.phi, js.phi_s2, p, cp, 0.0, P, P1, P2);
        if (js.fgam) spline_at(js.fgam, js.fgam_s2, p, cp, 0.0, F, t1, t2);
        J = jumps_from(p, g, P, P1, P2, F);
    }
    if (!(o[0] | o[1] | o[2] | o[3] | o[4] | o[5])) return 0.0;
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        if (!o[k]) continue;
        const double dx = p.lo + ni[k] * p.h - zx, dy = p.lo + nj[k] * p.h - zy;
        s += wk[k] * (J.v + dx * J.gx + dy * J.gy + 0.5 * (dx * dx * J.hxx + 2.0 * dx * dy * J.hxy + dy * dy * J.hyy));
    }
    return s;
}

__device__ __forceinline__ void stencil_nodes(const DevPlan& p, int cp, int (&ni)[6], int (&nj)[6]) {
    const int i0 = p.cp_i0[cp], j0 = p.cp_j0[cp], sxy = p.cp_sxy[cp];
    const int sx = (sxy & 1) ? 1 : -1, sy = (sxy & 2) ? 1 : -1;
    ni[0] = i0; nj[0] = j0;
    ni[1] = i0 + 1; nj[1] = j0;
    ni[2] = i0 - 1; nj[2] = j0;
    ni[3] = i0; nj[3] = j0 + 1;
    ni[4] = i0; nj[4] = j0 - 1;
    ni[5] = i0 + sx; nj[5] = j0 + sy;
}

__device__ inline double block_sum(double v, double* red) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    v = wave_allsum(v);
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
    for (int k = 0; k < nw; ++k) s += red[k];
    return s;
}

// ---------------------------------------------------------------- correction (Alg. 2)

// Correction of the right-hand side at irregular node r: for each arm to a
// neighbour across Gamma, the jump continued from the crossing along the arm by
// its second-order Taylor expansion, times -s_r / h^2.
__device__ inline double correction_at(const DevPlan& p, const JumpSrc& js, int r) {
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
            const J6 J = jumps_at(p, p.q_geo[k], js);
            v = J.v;
            g = ax ? J.gy : J.gx;
            hh = ax ? J.hyy : J.hxx;
        }
        acc -= s * (v + d * g + 0.5 * d * d * hh);
    }
    return acc * p.inv_h2;
}

// Samples cp0 .. cp0 + 63 (one per lane) by a workgroup of 16 wavefronts: the
// workgroup partials of the weighted sine sums (row g of `partial` holds
// workgroup g's sums for all M samples) are split over wavefronts 0..14, added
// in a fixed order; wavefront 15 makes the jump terms of the stencil nodes
// outside Omega, and wavefront 0 adds them and writes out[cp] (also to
// red[lane], for the caller).
// red: 16 x 64 doubles of LDS.  Returns false, having written nothing, while
// *skip is nonzero (skip may be null); the flag's latency overlaps the loads.
__device__ inline bool reduce_samples64(const DevPlan& p, const JumpSrc& js, const double* __restrict__ partial,
                                        int G, int cp0, double* __restrict__ out, double* red,
                                        const int* __restrict__ skip = nullptr) {
    __shared__ double outside[64];
    constexpr int kOutsideWave = 15;                    // makes the jump terms only
    constexpr int kRowWaves = 15, kRows = 18;           // rows wave + 15 k, k < 18, requested at once
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int cp = cp0 + lane, M = p.M;
    const int skipped = load_flag_or_zero(skip);
    double s = 0.0;
    if (cp < M) {
        if (wave == kOutsideWave) {
            int ni[6], nj[6];
            stencil_nodes(p, cp, ni, nj);
            outside[lane] = outside_terms(p, js, cp, ni, nj, p.cp_w + 6 * (size_t)cp);
        } else {
            // every row is loaded from a row that exists (then selected), so no
            // load waits under its own condition before the next is requested
            double r[kRows];
#pragma unroll
            for (int k = 0; k < kRows; ++k) {
                const int g = wave + kRowWaves * k;
                const double v = partial[(size_t)(g < G ? g : G - 1) * M + cp];
                r[k] = g < G ? v : 0.0;
            }
#pragma unroll
            for (int k = 0; k < kRows; ++k) s += r[k];
            for (int g = wave + kRowWaves * kRows; g < G; g += kRowWaves) s += partial[(size_t)g * M + cp];
        }
    }
    if (skipped) return false;                          // the same for the whole workgroup
    red[wave * 64 + lane] = s;
    __syncthreads();
    if (wave == 0 && cp < M) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < 16; ++w) t += red[w * 64 + lane];
        const double v = t * (2.0 / p.N) + outside[lane];
        out[cp] = v;
        red[lane] = v;                                  // left in LDS for the caller
    }
    __syncthreads();
    return true;
}

// ---------------------------------------------------------------- sparse fast solve, R modes per workgroup
//
// LDS of the sparse fast solve: the quarter sine table and R padded mode
// solutions (node i at i + (i - 1) / C, so the lanes' chunk-strided accesses
// fall in different banks).
struct ModesLds {
    double* sq;   // N/2 + 2
    double* xs;   // R x (N + 64)
    double* ex;   // R x kMaxExtra: sums of the extra pieces of long columns
};

template <int R>
__device__ __forceinline__ ModesLds modes_lds(double* smem, int N) {
    ModesLds L;
    L.sq = smem;
    L.xs = smem + (N / 2 + 2);
    L.ex = L.xs + (size_t)R * (N + 64);
    return L;
}

// Sine modes l = base + 1 .. base + R (those <= n) by a workgroup of
// kModeWaves wavefronts.
//  1. Sparse sine sums of the corrected right-hand side along y: wavefront w
//     walks sub-table w of the interleaved node table (each lane owns whole
//     columns); per node the sines of all R modes come from three table
//     lookups and the recurrence sin((l+1)t) = 2 cos t sin(lt) - sin((l-1)t),
//     and a column's R sums are stored when its last node is reached.
//  2. The tridiagonal solve along x of each mode (one wavefront per mode).
//  3. The weighted six-point gather at every sample (the row sines by the same
//     recurrence): emit(cp, s) with s the sum over the R modes, for
//     cp = tid, tid + 64 kModeWaves, ...
// L.sq must hold the sine table of p.N, or sinq (the table in device memory)
// is given and loaded here; must be called by the whole workgroup.  The round
// does nothing while *skip is nonzero (skip may be null); the flag is checked
// after the first requests and the clear, so its latency overlaps theirs.
template <int C, int R, class Emit>
__device__ __forceinline__ void modes_round(const DevPlan& p, const double* __restrict__ corr, int base,
                                            const ModesLds& L, Emit emit, const double* __restrict__ sinq = nullptr,
                                            const int* __restrict__ skip = nullptr) {
    constexpr int XS = 64 * (C + 1);
    constexpr int NT = kModeWaves * 64;
    const int N = p.N, n = p.n, M = p.M, mask2 = 2 * N - 1, half = N / 2;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const double* sq = L.sq;
    const int l0 = base + 1;
    const int nact = min(R, n - base);                  // modes of this round that exist
    const int skipped = load_flag_or_zero(skip);
    // the first rows of this wavefront's node table are requested before
    // anything waits, so their latency overlaps the table load and the clear;
    // the sub-table's bounds come with the plan's fields, not from memory
    const int wu = __builtin_amdgcn_readfirstlane(wave);
    int t_beg = p.sub_offv[0], t_end = p.sub_offv[1];  // multiples of kSlots
#pragma unroll
    for (int w = 1; w < kModeWaves; ++w)               // constant indices: loaded with the other fields
        if (wu == w) {
            t_beg = p.sub_offv[w];
            t_end = p.sub_offv[w + 1];
        }
    int pk[kSlots], pkn[kSlots];
    double cv[kSlots], cvn[kSlots];
    if (t_beg < t_end) {
#pragma unroll
        for (int q = 0; q < kSlots; ++q) {
            pk[q] = p.il_ij[(size_t)(t_beg + q) * 64 + lane];
            cv[q] = corr[(size_t)(t_beg + q) * 64 + lane];
        }
    }
    // also requested now: this wavefront's mode constants (phase 2) and the
    // stencil data of the thread's first kPre samples (phase 3)
    constexpr int kPre = 2;
    ModeConst mcw{};
    if (wave < nact) mcw = p.modes[l0 + wave];
    int4 pre_pk[kPre];
    double2 pre_w[kPre][3];
#pragma unroll
    for (int q = 0; q < kPre; ++q) {
        const int cp = tid + q * NT;
        if (cp < M) {
            pre_pk[q] = p.cp_pack[cp];
            const double2* w2 = reinterpret_cast<const double2*>(p.cp_w + 6 * (size_t)cp);
            pre_w[q][0] = w2[0];
            pre_w[q][1] = w2[1];
            pre_w[q][2] = w2[2];
        }
    }
    if (sinq)
        for (int k = tid; k <= N / 2; k += NT) L.sq[k] = sinq[k];
    for (int k = tid; k < R * XS; k += NT) L.xs[k] = 0.0;
    if (skipped) return;                                // the same for the whole workgroup
    __syncthreads();
    {
        double acc[R];
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] = 0.0;
        for (int t0 = t_beg; t0 < t_end; t0 += kSlots) {
            const bool more = t0 + kSlots < t_end;      // next group's loads overlap this group's sums
            if (more) {
#pragma unroll
                for (int q = 0; q < kSlots; ++q) {
                    pkn[q] = p.il_ij[(size_t)(t0 + kSlots + q) * 64 + lane];
                    cvn[q] = corr[(size_t)(t0 + kSlots + q) * 64 + lane];
                }
            }
            // sin((l0 + r) t), t = pi j / N, for r = 0 .. R-1: two table values,
            // then s_{r+1} = 2 cos t s_r - s_{r-1}.  The group's table values are
            // read before any of its sums is stored, so their latencies overlap
            double s0[kSlots], s1[kSlots], c2[kSlots];
#pragma unroll
            for (int q = 0; q < kSlots; ++q) {
                const int j = pk[q] & 0xfff;
                const int m0 = (int)(__umul24((unsigned)j, (unsigned)l0) & mask2);
                s0[q] = sinpi_n(sq, m0, N);
                s1[q] = R > 1 ? sinpi_n(sq, (m0 + j) & mask2, N) : 0.0;
                c2[q] = R > 2 ? 2.0 * sinpi_n(sq, (j + half) & mask2, N) : 0.0;
            }
#pragma unroll
            for (int q = 0; q < kSlots; ++q) {
                double sp = s0[q], sc = s1[q];
                acc[0] = fma(cv[q], sp, acc[0]);
                if (R > 1) acc[1] = fma(cv[q], sc, acc[1]);
#pragma unroll
                for (int r = 2; r < R; ++r) {
                    const double sn = fma(c2[q], sc, -sp);
                    acc[r] = fma(cv[q], sn, acc[r]);
                    sp = sc;
                    sc = sn;
                }
                if (pk[q] < 0) {                        // last node of its piece
                    const int dest = (pk[q] >> 16) & 0x7fff;
                    double* to = dest < kExtraFlag ? L.xs + dest : L.ex + (dest - kExtraFlag);
                    const int stride = dest < kExtraFlag ? XS : kMaxExtra;
                    if (nact == R) {
#pragma unroll
                        for (int r = 0; r < R; ++r) to[r * stride] = acc[r];
                    } else {
#pragma unroll
                        for (int r = 0; r < R; ++r)
                            if (r < nact) to[r * stride] = acc[r];
                    }
#pragma unroll
                    for (int r = 0; r < R; ++r) acc[r] = 0.0;
                }
            }
            if (more) {
#pragma unroll
                for (int q = 0; q < kSlots; ++q) {
                    pk[q] = pkn[q];
                    cv[q] = cvn[q];
                }
            }
        }
    }
    __syncthreads();
    // long columns: add their extra pieces in a fixed order
    for (int k = tid; k < p.n_split * R; k += NT) {
        const int c = k / R, r = k % R;
        if (r < nact) {
            const int pos = p.split[3 * c], e0 = p.split[3 * c + 1], ne = p.split[3 * c + 2];
            double v = L.xs[r * XS + pos];
            for (int e = 0; e < ne; ++e) v += L.ex[r * kMaxExtra + e0 + e];
            L.xs[r * XS + pos] = v;
        }
    }
    __syncthreads();
    static_assert(R <= kModeWaves, "one mode per wavefront at most");
    if (wave < nact) {
        double* x = L.xs + wave * XS;
        if constexpr (C > 32) {
            mode_solve_lds<C>(x, mcw, lane, N, p.h2);
        } else {
            double e[C];
#pragma unroll
            for (int c = 0; c < C; ++c) e[c] = x[lane * (C + 1) + 1 + c] * p.h2;
            mode_solve<C>(e, mcw, lane, N);
#pragma unroll
            for (int c = 0; c < C; ++c)
                if (lane < 63 || c < C - 1) x[lane * (C + 1) + 1 + c] = e[c];
        }
    }
    __syncthreads();
    auto gather = [&](int cp, const int4 pk4, const double2 wa, const double2 wb, const double2 wc) {
        const int i0 = pk4.x, j0 = pk4.y, sxy = pk4.z;
        const int sx = (sxy & 1) ? 1 : -1;
        const bool syp = (sxy & 2) != 0;
        const double w0 = wa.x, wE = wa.y, wW = wb.x, wN = wb.y, wS = wc.x, wD = wc.y;
        // places of the stencil columns in the padded layout (node 0 lies on
        // the box: zero); the sine arguments advance by j per mode
        const int pc = i0 + (i0 - 1) / C, pe = i0 + i0 / C + 1, pw = i0 > 1 ? i0 - 1 + (i0 - 2) / C : -1;
        // sines of the rows j0, j0 + 1, j0 - 1 for the modes l0 + q: two table
        // values each, then the three-term recurrence in q
        const int a0 = (int)(__umul24((unsigned)j0, (unsigned)l0) & mask2);
        const int ap = (int)(__umul24((unsigned)(j0 + 1), (unsigned)l0) & mask2);
        const int am = (int)(__umul24((unsigned)(j0 - 1), (unsigned)l0) & mask2);
        double s0p = sinpi_n(sq, a0, N), spp = sinpi_n(sq, ap, N), smp = sinpi_n(sq, am, N);
        double s0c = 0.0, spc = 0.0, smc = 0.0, c0 = 0.0, cpl = 0.0, cmi = 0.0;
        if (R > 1) {
            s0c = sinpi_n(sq, (a0 + j0) & mask2, N);
            spc = sinpi_n(sq, (ap + j0 + 1) & mask2, N);
            smc = sinpi_n(sq, (am + j0 - 1) & mask2, N);
        }
        if (R > 2) {
            c0 = 2.0 * sinpi_n(sq, (j0 + half) & mask2, N);
            cpl = 2.0 * sinpi_n(sq, (j0 + 1 + half) & mask2, N);
            cmi = 2.0 * sinpi_n(sq, (j0 - 1 + half) & mask2, N);
        }
        double s = 0.0;
        // modes beyond n were never written: their solutions are zero
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const double* xq = L.xs + q * XS;
            double s0, sp, sm;
            if (q == 0) {
                s0 = s0p;
                sp = spp;
                sm = smp;
            } else if (q == 1) {
                s0 = s0c;
                sp = spc;
                sm = smc;
            } else {
                s0 = fma(c0, s0c, -s0p);
                sp = fma(cpl, spc, -spp);
                sm = fma(cmi, smc, -smp);
                s0p = s0c;
                spp = spc;
                smp = smc;
                s0c = s0;
                spc = sp;
                smc = sm;
            }
            const double xc = xq[pc];
            const double xe = xq[pe];
            const double xw = pw >= 0 ? xq[pw] : 0.0;
            const double xd = sx > 0 ? xe : xw;
            s += s0 * (w0 * xc + wE * xe + wW * xw) + sp * wN * xc + sm * wS * xc + (syp ? sp : sm) * wD * xd;
        }
        emit(cp, s);
    };
#pragma unroll
    for (int q = 0; q < kPre; ++q) {
        const int cp = tid + q * NT;
        if (cp < M) gather(cp, pre_pk[q], pre_w[q][0], pre_w[q][1], pre_w[q][2]);
    }
    for (int cp = tid + kPre * NT; cp < M; cp += NT) {
        const double2* w2 = reinterpret_cast<const double2*>(p.cp_w + 6 * (size_t)cp);
        gather(cp, p.cp_pack[cp], w2[0], w2[1], w2[2]);
    }
    __syncthreads();
}

}  // namespace kfbi
