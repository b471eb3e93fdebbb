// Restarted GMRES (Alg. 5) on the boundary density, resident on the device.
//
// One step of the iteration follows one K_D apply (whose output is b.w) and is
// five launches, so that the vector work is spread over many workgroups:
//   dots1   per chunk: mode 0: phi <- xcur (the iterate the apply was given),
//           z = ghat - w and partial |z|^2; mode 1: partial dots V_i . w, i <= j
//   upd1    per chunk: h_i = sum of the partials; z = w - sum h_i V_i; partial
//           dots V_i . z (classical Gram-Schmidt, second pass)
//   upd2    per chunk: z -= sum h'_i V_i; partial |z|^2
//   commit  one workgroup: the new Hessenberg column, the Givens rotations and
//           the residual estimate (mode 1), or the true residual (mode 0);
//           the state transition; at the end of a cycle the triangular solve
//   emit    per chunk: the next K_D input (new basis vector, or the updated
//           iterate at the end of a cycle) and its spline second derivatives.
// Partial sums are added in a fixed order, so results do not depend on timing.
// Only commit writes the state, and it runs alone (one workgroup); every other
// launch only reads it.
#pragma once

#include "device.h"

namespace kfbi {

constexpr int kGmChunk = 256;            // vector elements per workgroup (one per thread)
constexpr int kGmHalo = kSplineK + 1;    // reach of the spline filter on each side

enum GmKind { kGmNewCycle = 0, kGmNextVector = 1, kGmCycleEnd = 2, kGmDone = 3 };

__host__ __device__ inline int gm_chunks(int M) { return (M + kGmChunk - 1) / kGmChunk; }
// doubles of partial sums a problem needs: two dot blocks of (m+1) x gc, one norm block of gc
__host__ __device__ inline size_t gm_part_size(int m, int gc) { return (size_t)(2 * (m + 1) + 1) * gc; }

__device__ inline double gm_block_sum(double v, double* red) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    return red[0] + red[1] + red[2] + red[3];
}

// Partial dots of the chunk with V_0..V_j: x[q] is the vector at element
// c0 + lane + 64 q.  Wave w takes i = w, w + 4, ...
__device__ inline void gm_chunk_dots(const double* __restrict__ V, const double (&x)[4], int M, int c, int gc,
                                     int j, double* __restrict__ out) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int c0 = c * kGmChunk;
    for (int i = wave; i <= j; i += 4) {
        const double* Vi = V + (size_t)i * M + c0;
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int t = lane + 64 * q;
            if (c0 + t < M) s = fma(Vi[t], x[q], s);
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
        if (lane == 0) out[(size_t)i * gc + c] = s;
    }
}

__device__ inline void gm_dots1(const GmresBufs& b, int M, int c) {
    __shared__ double red[4];
    const GmresState* st = b.st;
    const int mode = st->mode;
    if (mode == 2) return;
    const int tid = threadIdx.x, lane = tid & 63, gc = b.gc, m = b.m;
    const int c0 = c * kGmChunk, e = c0 + tid;
    if (mode == 0) {
        double r = 0.0;
        if (e < M) {
            b.phi[e] = b.xcur[e];
            r = b.ghat[e] - b.w[e];
            b.z[e] = r;
        }
        const double s = gm_block_sum(r * r, red);
        if (tid == 0) b.part[(size_t)2 * (m + 1) * gc + c] = s;
        return;
    }
    double x[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int t = c0 + lane + 64 * q;
        x[q] = t < M ? b.w[t] : 0.0;
    }
    gm_chunk_dots(b.V, x, M, c, gc, st->j, b.part);
}

// pass 0: z = w - sum h_i V_i and the second-pass dots; pass 1: z -= sum h'_i V_i and |z|^2
__device__ inline void gm_update(const GmresBufs& b, int M, int c, int pass) {
    __shared__ double hs[kMaxRestart + 2];
    __shared__ double zs[kGmChunk];
    __shared__ double red[4];
    const GmresState* st = b.st;
    if (st->mode != 1) return;
    const int tid = threadIdx.x, lane = tid & 63, gc = b.gc, m = b.m, j = st->j;
    const double* coef = b.part + (pass == 0 ? 0 : (size_t)(m + 1) * gc);
    for (int i = tid; i <= j; i += kGmChunk) {
        double s = 0.0;
        for (int cc = 0; cc < gc; ++cc) s += coef[(size_t)i * gc + cc];
        hs[i] = s;
    }
    __syncthreads();
    const int c0 = c * kGmChunk, e = c0 + tid;
    double zv = 0.0;
    if (e < M) {
        double a = pass == 0 ? b.w[e] : b.z[e];
        for (int i0 = 0; i0 <= j; i0 += 8) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = i0 + u <= j ? b.V[(size_t)(i0 + u) * M + e] : 0.0;
#pragma unroll
            for (int u = 0; u < 8; ++u) a -= (i0 + u <= j ? hs[i0 + u] : 0.0) * v[u];
        }
        zv = a;
        b.z[e] = a;
    }
    if (pass == 0) {
        zs[tid] = zv;
        __syncthreads();
        double x[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) x[q] = zs[lane + 64 * q];
        gm_chunk_dots(b.V, x, M, c, gc, j, b.part + (size_t)(m + 1) * gc);
    } else {
        const double s = gm_block_sum(zv * zv, red);
        if (tid == 0) b.part[(size_t)2 * (m + 1) * gc + c] = s;
    }
}

// One workgroup of kGmChunk threads.
__device__ inline void gm_commit(const GmresBufs& b) {
    __shared__ double red[4];
    __shared__ double col[kMaxRestart + 2];
    __shared__ double cs_s[kMaxRestart], sn_s[kMaxRestart];
    __shared__ double Hs[kMaxRestart * (kMaxRestart + 1)];
    __shared__ int s_end;
    GmresState* st = b.st;
    const int mode = st->mode;
    if (mode == 2) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m = b.m, gc = b.gc, j = st->j, it = st->it, first = st->first, max_iter = st->max_iter;
    const double r0_in = st->r0, tol = st->tol;
    const double* norm = b.part + (size_t)2 * (m + 1) * gc;
    double v = 0.0;
    for (int cc = tid; cc < gc; cc += kGmChunk) v += norm[cc];
    const double nrm = sqrt(gm_block_sum(v, red));
    if (mode == 0) {
        if (tid == 0) {
            const double beta = nrm;
            const double r0 = first ? beta : r0_in;
            const double rel = r0 > 0.0 ? beta / r0 : 0.0;
            const bool done = r0 == 0.0 || beta == 0.0 || rel < tol || it >= max_iter;
            st->r0 = r0;
            st->first = 0;
            st->relres = rel;
            if (done) {
                st->converged = (r0 == 0.0 || beta == 0.0 || rel < tol) ? 1 : -1;
                st->mode = 2;
                st->kind = kGmDone;
            } else {
                b.g[0] = beta;
                for (int k = 1; k <= m; ++k) b.g[k] = 0.0;
                st->j = 0;
                st->mode = 1;
                st->cycles += 1;
                st->kind = kGmNewCycle;
                st->scale = 1.0 / beta;
            }
        }
        return;
    }
    // mode 1: column j of the Hessenberg matrix from the two Gram-Schmidt passes
    const double* d1 = b.part;
    const double* d2 = b.part + (size_t)(m + 1) * gc;
    for (int i = tid; i <= j; i += kGmChunk) {
        double s1 = 0.0, s2 = 0.0;
        for (int cc = 0; cc < gc; ++cc) {
            s1 += d1[(size_t)i * gc + cc];
            s2 += d2[(size_t)i * gc + cc];
        }
        col[i] = s1 + s2;
    }
    if (tid < j) {
        cs_s[tid] = b.cs[tid];
        sn_s[tid] = b.sn[tid];
    }
    __syncthreads();
    if (tid == 0) {
        const double hn = nrm;
        double a = col[0];
        for (int i = 0; i < j; ++i) {
            const double cn = col[i + 1], cc = cs_s[i], ss = sn_s[i];
            col[i] = cc * a + ss * cn;
            a = -ss * a + cc * cn;
        }
        const double den = hypot(a, hn);
        const double cs = den > 0.0 ? a / den : 1.0;
        const double sn = den > 0.0 ? hn / den : 0.0;
        col[j] = den;
        col[j + 1] = 0.0;
        b.cs[j] = cs;
        b.sn[j] = sn;
        const double gj = b.g[j];
        b.g[j + 1] = -sn * gj;
        b.g[j] = cs * gj;
        const int jn = j + 1, itn = it + 1;
        const double est = fabs(sn * gj) / r0_in;
        st->relres = est;
        st->it = itn;
        const bool end = est < tol || jn == m || itn >= max_iter || hn == 0.0;
        s_end = end ? 1 : 0;
        st->jn = jn;
        if (end) {
            st->mode = 0;
            st->kind = kGmCycleEnd;
        } else {
            st->j = jn;
            st->kind = kGmNextVector;
            st->scale = hn > 0.0 ? 1.0 / hn : 0.0;
        }
    }
    __syncthreads();
    double* Hj = b.H + (size_t)j * (m + 1);
    if (tid <= j + 1) Hj[tid] = col[tid];
    if (!s_end) return;
    // end of the cycle: H[0:jn, 0:jn] y = g[0:jn], one wavefront, column by column
    const int jn = j + 1;
    for (int t = tid; t < jn * (m + 1); t += kGmChunk) {
        const int kc = t / (m + 1), i = t % (m + 1);
        Hs[t] = kc == j ? col[i] : b.H[t];
    }
    __syncthreads();
    if (wave == 0) {
        double gk = lane < jn ? b.g[lane] : 0.0;
        double yk = 0.0;
        for (int i = jn - 1; i >= 0; --i) {
            const double yi = __shfl(gk, i, 64) / Hs[i * (m + 1) + i];
            if (lane == i) yk = yi;
            if (lane < i) gk -= Hs[i * (m + 1) + lane] * yi;
        }
        if (lane < jn) b.y[lane] = yk;
    }
}

// The next K_D input for elements of chunk c, and its spline second derivatives
// (the filter reads kGmHalo neighbours on each side, wrapping around Gamma).
__device__ inline void gm_emit(const DevPlan& p, const GmresBufs& b, int M, int c) {
    __shared__ double win[kGmChunk + 2 * kGmHalo];
    const GmresState* st = b.st;
    const int kind = st->kind;
    if (kind == kGmDone) return;
    const int tid = threadIdx.x, c0 = c * kGmChunk;
    const double scale = st->scale;
    const int jn = st->jn;
    for (int k = tid; k < kGmChunk + 2 * kGmHalo; k += kGmChunk) {
        int e = (c0 - kGmHalo + k) % M;
        if (e < 0) e += M;
        double x;
        if (kind == kGmCycleEnd) {
            x = b.phi[e];
            for (int i = 0; i < jn; ++i) x = fma(b.y[i], b.V[(size_t)i * M + e], x);
        } else {
            x = b.z[e] * scale;
        }
        win[k] = x;
    }
    __syncthreads();
    const int e = c0 + tid;
    if (e >= M) return;
    const double x = win[kGmHalo + tid];
    if (kind == kGmNewCycle) b.V[e] = x;
    if (kind == kGmNextVector) b.V[(size_t)st->j * M + e] = x;
    b.xcur[e] = x;
    constexpr int K = kSplineK;
    double s = 0.0;
#pragma unroll
    for (int q = -K - 1; q <= K + 1; ++q) s = fma(p.taps[q + K + 1], win[kGmHalo + tid + q], s);
    b.s2cur[e] = s;
}

}  // namespace kfbi
