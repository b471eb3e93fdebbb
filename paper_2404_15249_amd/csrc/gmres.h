// Restarted GMRES (Alg. 5) on the boundary density, resident on the device.
//
// One step of the iteration follows one K_D apply and takes, besides it, two
// launches, so the vector work is spread over many workgroups:
//   dots1   fused into the apply's last launch (reduce_samples64), per 64
//           samples: mode 0: phi <- xcur (the iterate the apply was given),
//           z = ghat - w and partial |z|^2; mode 1: partial dots V_i . w, i <= j
//   upd1    per chunk of kGmChunk: h_i = sum of the partials; z = w - sum h_i
//           V_i; partial |z|^2 and |w|^2.  The workgroup that finishes last (an
//           atomic count, no waiting) commits.  Classical Gram-Schmidt keeps
//           the new vector orthogonal to the basis to about eps |w| / |z|; only
//           when |z| < reorth |w| (1e-3 by default) does that workgroup first
//           make a second pass over the whole vector itself.  For these
//           second-kind operators the cancellation stays far above that bound.
//   commit  the new Hessenberg column, the Givens rotations and the residual
//           estimate (mode 1) or the true residual (mode 0), the state
//           transition, and at the end of a cycle the triangular solve
//   emit    per chunk: the next K_D input (new basis vector, or the updated
//           iterate at the end of a cycle) and its spline second derivatives.
// Partial sums are added in a fixed order, so results do not depend on timing.
// Only commit writes the state, and it runs after every other workgroup of its
// launch has read it.
#pragma once

#include "device.h"

namespace kfbi {

constexpr int kGmChunk = 256;            // vector elements per workgroup (one per thread)
constexpr int kGmHalo = kSplineK + 1;    // reach of the spline filter on each side

enum GmKind { kGmNewCycle = 0, kGmNextVector = 1, kGmCycleEnd = 2, kGmDone = 3 };

// GmresState::converged when a norm of the iteration came out NaN or Inf
constexpr int kGmNonfinite = -2;

__host__ __device__ inline int gm_chunks(int M) { return (M + kGmChunk - 1) / kGmChunk; }
__host__ __device__ inline int gm_chunks64(int M) { return (M + 63) / 64; }
// doubles of partial sums a problem needs: first-pass dots (m+1) x gc64, norms
// of the update (gc), of the residual (gc64) and of the apply's output (gc)
__host__ __device__ inline size_t gm_part_size(int m, int gc, int gc64) {
    return (size_t)(m + 1) * gc64 + 2 * gc + gc64;
}

struct GmPart {
    double* d1;     // [i * gc64 + c64]
    double* nrm;    // [c]
    double* nrm0;   // [c64]
    double* nrmw;   // [c]: |w|^2 of the chunk (first update)
};
__device__ __forceinline__ GmPart gm_part(const GmresBufs& b) {
    GmPart q;
    q.d1 = b.part;
    q.nrm = q.d1 + (size_t)(b.m + 1) * b.gc64;
    q.nrm0 = q.nrm + b.gc;
    q.nrmw = q.nrm0 + b.gc64;
    return q;
}

// The state an update launch works from, read once at its start: only the
// commit writes the state, after every workgroup of the launch has read it.
struct GmSnap {
    int mode, j, it, first, max_iter;
    double r0, tol, reorth;
};
__device__ __forceinline__ GmSnap gm_snap(const GmresState* st) {
    GmSnap s;
    s.mode = st->mode;
    s.j = st->j;
    s.it = st->it;
    s.first = st->first;
    s.max_iter = st->max_iter;
    s.r0 = st->r0;
    s.tol = st->tol;
    s.reorth = st->reorth;
    return s;
}

// The state, copied to the host-visible mirror (pinned host memory, null when
// there is none) by the thread that just wrote it: the host reads the mirror
// after a stream wait instead of copying the state back.
__device__ __forceinline__ void gm_publish(const GmresBufs& b) {
    if (b.pub) *b.pub = *b.st;
}

// What an emit launch takes from the state, given directly by the launch that
// starts a run (which writes the state itself): the kind, the scale, the
// source of the next input (x = xsrc * scale) and, when the run ends with
// x = 0 right away, where that zero goes.
struct EmitCtl {
    int kind;
    double scale;
    const double* xsrc;
    double* xzero;
};

// What the commit of an Arnoldi step reads besides the norms: the first-pass
// coefficients, the previous rotations and g_j.  Every workgroup of the update
// loads them beside its basis values (none changes before the commit), so the
// one that commits has them at hand.
struct GmCommitIn {
    double h1[kMaxRestart + 2];
    double cs[kMaxRestart], sn[kMaxRestart];
    double gj;
};

__device__ __forceinline__ double wave_sum(double v) { return wave_allsum(v); }

__device__ inline double gm_block_sum(double v, double* red) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    v = wave_allsum(v);
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    return red[0] + red[1] + red[2] + red[3];
}

// Sums over the wavefront of G values per lane at once: log2(G) halving steps
// (each lane keeps half of its values and adds its partner's other half), then
// plain butterfly steps.  Returns the wavefront sum of value number
// (lane >> (6 - log2 G)) & (G - 1); 64 / G lanes hold each sum.
template <int G>
__device__ __forceinline__ double wave_sum_many(double (&p)[G]) {
    static_assert(G >= 2 && G <= 64 && (G & (G - 1)) == 0, "G must be a power of two");
    const int lane = threadIdx.x & 63;
    int off = 32;
#pragma unroll
    for (int half = G / 2; half >= 1; half /= 2, off >>= 1) {
        const bool hi = (lane & off) != 0;
#pragma unroll
        for (int u = 0; u < half; ++u) {
            // the empty asm makes both operands register values: otherwise the
            // compiler turns "hi ? p[a] : p[b]" into p[hi ? a : b], a run-time
            // index into the array that it lowers to a chain of G selects
            double lo_v = p[u], hi_v = p[u + half];
            asm volatile("" : "+v"(lo_v), "+v"(hi_v));
            const double keep = hi ? hi_v : lo_v;
            const double send = hi ? lo_v : hi_v;
            p[u] = keep + __shfl_xor(send, off, 64);
        }
    }
    for (; off >= 1; off >>= 1) p[0] += __shfl_xor(p[0], off, 64);
    return p[0];
}

// Loads V_i at element e (0 outside [0, M) and for i > j) for i < 4 * 16,
// grouped by 16.
__device__ __forceinline__ void gm_load_basis(const double* __restrict__ V, int M, int e, int j, double (&v)[4][16]) {
    const bool in = e < M;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int i = 16 * g + u;
            v[g][u] = (in && i <= j) ? V[(size_t)i * M + e] : 0.0;
        }
    }
}

// The basis values the first pass needs from this wavefront (V_i at its lane's
// sample for i = wave, wave + 16, ...; kMaxRestart <= 64), requested before the
// apply's reduction so that their latency overlaps it.  Every row that can be
// in use (i < m) is requested without waiting for the state; rows past the
// current column are not used.
// Wavefront 0 also requests what a residual step reads: the iterate the apply
// was given and ghat at its lane's sample.
struct GmPre {
    double v[4];
    double xc, gh;
};
__device__ __forceinline__ GmPre gm_dots1_prefetch(const GmresBufs& b, int M, int c64) {
    static_assert(kMaxRestart <= 64, "four basis values per lane");
    GmPre pre;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, cp = c64 * 64 + lane;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int i = wave + 16 * k;
        pre.v[k] = (i < b.m && cp < M) ? b.V[(size_t)i * M + cp] : 0.0;
    }
    pre.xc = pre.gh = 0.0;
    if (wave == 0 && cp < M) {
        pre.xc = b.xcur[cp];
        pre.gh = b.ghat[cp];
    }
    return pre;
}

// First step of GMRES on samples c64 * 64 .. + 63, called by a workgroup of 16
// wavefronts right after it computed w there (wv[lane] in LDS); pre: the
// values from gm_dots1_prefetch (null: loaded here); mode, j: the state's, as
// read by the caller at its start.
__device__ inline void gm_dots1_64(const GmresBufs& b, int M, int c64, const double* wv, const GmPre* pre, int mode,
                                   int j) {
    if (mode == 2) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int cp = c64 * 64 + lane;
    const GmPart q = gm_part(b);
    if (mode == 0) {
        if (wave != 0) return;
        double r = 0.0;
        if (cp < M) {
            const double xc = pre ? pre->xc : b.xcur[cp], gh = pre ? pre->gh : b.ghat[cp];
            b.phi[cp] = xc;
            r = gh - wv[lane];
            b.z[cp] = r;
        }
        const double s = wave_sum(r * r);
        if (lane == 0) q.nrm0[c64] = s;
        return;
    }
    const int gc64 = b.gc64;
    const double x = cp < M ? wv[lane] : 0.0;
    if (pre) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int i = wave + 16 * k;
            if (i <= j) {
                const double s = wave_sum(cp < M ? pre->v[k] * x : 0.0);
                if (lane == 0) q.d1[(size_t)i * gc64 + c64] = s;
            }
        }
        return;
    }
    for (int i = wave; i <= j; i += 16) {
        const double s = wave_sum(cp < M ? b.V[(size_t)i * M + cp] * x : 0.0);
        if (lane == 0) q.d1[(size_t)i * gc64 + c64] = s;
    }
}
__device__ inline void gm_dots1_64(const GmresBufs& b, int M, int c64, const double* wv) {
    gm_dots1_64(b, M, c64, wv, nullptr, b.st->mode, b.st->j);
}

// What one update workgroup loads, requested before the state is known: the
// basis values at its element for every row that can be in use (i < m; rows
// past the current column are loaded and not used), w, and per thread i < m
// row i's first-pass dot partials summed, the rotation (c_i, s_i) and g_i.
struct GmUpdIn {
    double v[4][16];
    double w;
    double h, cs, sn, g;
};
// Chunk counts up to which one thread adds a row of partials (or the chunk
// norms) itself; above them (the surface problem's long vectors) the
// workgroup's threads split the work, so the chain of dependent loads stays short.
constexpr int kGmSerialSums = 32;

// h_i = the sum of row i of the nco chunk partials, i < m, for many chunks:
// kGmChunk / m threads per row, each adding every (kGmChunk / m)-th chunk in
// order, then the parts added in order.  Returns h_tid for tid < m; the same
// order in every workgroup, so they all agree.  Called by the whole workgroup.
__device__ inline double gm_dots_spread(const double* d1, int m, int nco) {
    __shared__ double part[kGmChunk];
    const int tid = threadIdx.x, P = kGmChunk / m;
    double s = 0.0;
    if (tid < m * P) {
        const int i = tid / P, r = tid - i * P;
        const double* row = d1 + (size_t)i * nco;
        for (int c0 = r; c0 < nco; c0 += 16 * P) {
            double v[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) v[u] = c0 + u * P < nco ? row[c0 + u * P] : 0.0;   // issued together
#pragma unroll
            for (int u = 0; u < 16; ++u) s += v[u];
        }
    }
    part[tid] = s;
    __syncthreads();
    double h = 0.0;
    if (tid < m)
        for (int r = 0; r < P; ++r) h += part[tid * P + r];
    return h;
}

__device__ __forceinline__ GmUpdIn gm_update_loads(const GmresBufs& b, int M, int c) {
    const int tid = threadIdx.x, m = b.m, nco = b.gc64;
    const GmPart q = gm_part(b);
    const int e = c * kGmChunk + tid;
    GmUpdIn u;
    gm_load_basis(b.V, M, e, m - 1, u.v);
    u.w = e < M ? b.w[e] : 0.0;
    u.h = u.cs = u.sn = u.g = 0.0;
    if (tid < m) {
        u.cs = b.cs[tid];
        u.sn = b.sn[tid];
        u.g = b.g[tid];
    }
    if (nco <= kGmSerialSums) {
        if (tid < m) {
            double sum = 0.0;
#pragma unroll 16
            for (int cc = 0; cc < nco; ++cc) sum += q.d1[(size_t)tid * nco + cc];   // loads issued together
            u.h = sum;
        }
    } else {
        u.h = gm_dots_spread(q.d1, m, nco);
    }
    return u;
}

// The first Gram-Schmidt pass on chunk c from the loads above: h_i (into
// ci.h1, with the commit's other operands), z = w - sum h_i V_i, and the
// chunk's |z|^2 and |w|^2.
__device__ __forceinline__ void gm_update(const GmresBufs& b, int M, int c, int j, const GmUpdIn& u, GmCommitIn& ci,
                                          double* red) {
    const int tid = threadIdx.x;
    const GmPart q = gm_part(b);
    const int e = c * kGmChunk + tid;
    if (tid <= j) ci.h1[tid] = u.h;
    if (tid < j) {
        ci.cs[tid] = u.cs;
        ci.sn[tid] = u.sn;
    }
    if (tid == j) ci.gj = u.g;
    __syncthreads();
    double a = u.w;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        if (16 * g <= j) {
#pragma unroll
            for (int k = 0; k < 16; ++k)
                if (16 * g + k <= j) a -= ci.h1[16 * g + k] * u.v[g][k];
        }
    }
    if (e < M) b.z[e] = a;
    const double sz = gm_block_sum(a * a, red);
    const double sw = gm_block_sum(u.w * u.w, red);
    if (tid == 0) {
        q.nrm[c] = sz;
        q.nrmw[c] = sw;
    }
}

// Commit of a residual step (mode 0), by one workgroup of kGmChunk threads:
// beta = |ghat - K phi| from the partials the apply's reduction left, then the
// end of the solve or a new cycle.
__device__ inline void gm_commit_residual(const GmresBufs& b, const GmSnap& s, double* red) {
    const int tid = threadIdx.x, m = b.m;
    const GmPart q = gm_part(b);
    double v = 0.0;
    for (int cc = tid; cc < b.gc64; cc += kGmChunk) v += q.nrm0[cc];
    const double beta = sqrt(gm_block_sum(v, red));
    if (tid != 0) return;
    GmresState* st = b.st;
    if (!isfinite(beta)) {                                 // NaN or Inf in the data: stop here
        st->converged = kGmNonfinite;
        st->mode = 2;
        st->kind = kGmDone;
        gm_publish(b);
        return;
    }
    st->res_applies += 1;
    const double r0 = s.first ? beta : s.r0;
    const double rel = r0 > 0.0 ? beta / r0 : 0.0;
    const bool done = r0 == 0.0 || beta == 0.0 || rel < s.tol || s.it >= s.max_iter;
    st->r0 = r0;
    st->first = 0;
    st->relres = rel;
    if (done) {
        st->converged = (r0 == 0.0 || beta == 0.0 || rel < s.tol) ? 1 : -1;
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
    gm_publish(b);
}

// Commit of an Arnoldi step (mode 1), by one workgroup of kGmChunk threads:
// column j of the Hessenberg matrix (h1 + h2 from the two Gram-Schmidt
// passes, h_{j+1,j} = hn), the previous rotations down it and a new one, the
// residual estimate, the state transition, and at the end of a cycle the
// triangular solve.
__device__ inline void gm_commit_arnoldi(const GmresBufs& b, const GmSnap& s, const GmCommitIn& ci,
                                         const double* h2, double hn) {
    __shared__ double col[kMaxRestart + 2];
    __shared__ double rot[kMaxRestart];
    __shared__ double Hs[kMaxRestart * (kMaxRestart + 1)];
    __shared__ int s_end;
    GmresState* st = b.st;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m = b.m, j = s.j;
    if (tid <= j) col[tid] = ci.h1[tid] + h2[tid];
    __syncthreads();
    if (tid == 0) {
        // previous rotations down the column, eight at a time: their operands
        // are read together; the rotated entries go to rot[]
        double a = col[0];
        for (int i0 = 0; i0 < j; i0 += 8) {
            double cn[8], c8[8], s8[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const bool in = i0 + u < j;
                cn[u] = in ? col[i0 + u + 1] : 0.0;
                c8[u] = in ? ci.cs[i0 + u] : 1.0;
                s8[u] = in ? ci.sn[i0 + u] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                if (i0 + u < j) {
                    rot[i0 + u] = c8[u] * a + s8[u] * cn[u];
                    a = -s8[u] * a + c8[u] * cn[u];
                }
            }
        }
        for (int i = 0; i < j; ++i) col[i] = rot[i];
        const double den = hypot(a, hn);
        if (!isfinite(den) || !isfinite(ci.gj)) {         // NaN or Inf in the data: stop here
            st->converged = kGmNonfinite;
            st->mode = 2;
            st->kind = kGmDone;
            gm_publish(b);
            s_end = -1;
        } else {
            const double cs = den > 0.0 ? a / den : 1.0;
            const double sn = den > 0.0 ? hn / den : 0.0;
            col[j] = den;
            col[j + 1] = 0.0;
            b.cs[j] = cs;
            b.sn[j] = sn;
            const double gj = ci.gj;
            b.g[j + 1] = -sn * gj;
            b.g[j] = cs * gj;
            const int jn = j + 1, itn = s.it + 1;
            const double est = fabs(sn * gj) / s.r0;
            st->relres = est;
            st->it = itn;
            const bool end = est < s.tol || jn == m || itn >= s.max_iter || hn == 0.0;
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
    }
    __syncthreads();
    if (s_end < 0) return;
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
            const double yi = readlane_f64(gk, i) / Hs[i * (m + 1) + i];   // i is the same in every lane
            if (lane == i) yk = yi;
            if (lane < i) gk -= Hs[i * (m + 1) + lane] * yi;
        }
        if (lane < jn) b.y[lane] = yk;
    }
}

// Whether this workgroup finished the problem's last chunk of the launch (an
// atomic count of finished chunks; nobody waits); the last one resets the
// count for the next launch.  Called by the whole workgroup after its writes.
__device__ inline bool gm_last_chunk(const GmresBufs& b, int* s_last) {
    // every wavefront's stores (z, which a second pass of the committing
    // workgroup reads) complete before thread 0's fence publishes them: the
    // workgroup barrier alone does not wait for them
    __builtin_amdgcn_s_waitcnt(0x0F70);                    // vmcnt(0) (expcnt, lgkmcnt not waited)
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();                                   // this chunk's partials before the count
        const unsigned done = atomicAdd(b.cnt, 1u) + 1;
        *s_last = done == (unsigned)b.gc;
        if (*s_last) {
            __hip_atomic_store(b.cnt, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __threadfence();                               // the other chunks' partials after it
        }
    }
    __syncthreads();
    return *s_last != 0;
}

// The second Gram-Schmidt pass over the whole vector by the one workgroup that
// commits (only when the first pass cancelled below the threshold): h2 = V^T z
// in groups of sixteen basis vectors, z -= V h2; returns the new |z|^2.  h2
// goes to h2s (LDS).
__device__ inline double gm_second_pass(const GmresBufs& b, int M, int j, double* h2s, double* red) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        if (16 * g <= j) {
            double p[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) p[u] = 0.0;
            for (int e = tid; e < M; e += kGmChunk) {
                const double ze = b.z[e];
#pragma unroll
                for (int u = 0; u < 16; ++u)
                    if (16 * g + u <= j) p[u] = fma(b.V[(size_t)(16 * g + u) * M + e], ze, p[u]);
            }
            const double s = wave_sum_many<16>(p);
            if ((lane & 3) == 0) red[wave * 16 + (lane >> 2)] = s;
            __syncthreads();
            if (tid < 16) h2s[16 * g + tid] = 16 * g + tid <= j ? red[tid] + red[16 + tid] + red[32 + tid] + red[48 + tid] : 0.0;
            __syncthreads();
        }
    }
    double zz = 0.0;
    for (int e = tid; e < M; e += kGmChunk) {
        double a = b.z[e];
        for (int i = 0; i <= j; ++i) a -= h2s[i] * b.V[(size_t)i * M + e];
        b.z[e] = a;
        zz = fma(a, a, zz);
    }
    return gm_block_sum(zz, red);
}

// upd1 on chunk c; the workgroup that finishes the problem's last chunk then
// commits: a residual step (mode 0) from the residual's norm partials, an
// Arnoldi step (mode 1) from the first pass, after a second pass of its own
// when |z| < reorth |w|.
__device__ inline void gm_update1_commit(const GmresBufs& b, int M, int c) {
    __shared__ int s_last;
    __shared__ int s_second;
    __shared__ double s_zz;
    __shared__ double h2s[kMaxRestart + 2];
    __shared__ double red[64];
    __shared__ GmCommitIn ci;
    const GmUpdIn u = gm_update_loads(b, M, c);
    const GmSnap s = gm_snap(b.st);
    if (s.mode == 2) return;
    if (s.mode == 1) gm_update(b, M, c, s.j, u, ci, red);
    if (!gm_last_chunk(b, &s_last)) return;
    if (s.mode == 0) {
        gm_commit_residual(b, s, red);
        return;
    }
    for (int i = threadIdx.x; i < kMaxRestart + 2; i += kGmChunk) h2s[i] = 0.0;
    if (b.gc <= kGmSerialSums) {
        if (threadIdx.x == 0) {
            const GmPart q = gm_part(b);
            double zz = 0.0, ww = 0.0;
#pragma unroll 8
            for (int cc = 0; cc < b.gc; ++cc) {            // fixed order
                zz += q.nrm[cc];
                ww += q.nrmw[cc];
            }
            s_second = zz < s.reorth * s.reorth * ww;
            s_zz = zz;
        }
    } else {                                               // many chunks: every thread, then a block sum
        const GmPart q = gm_part(b);
        double a = 0.0, w = 0.0;
        for (int cc = threadIdx.x; cc < b.gc; cc += kGmChunk) {
            a += q.nrm[cc];
            w += q.nrmw[cc];
        }
        const double zz = gm_block_sum(a, red), ww = gm_block_sum(w, red);
        if (threadIdx.x == 0) {
            s_second = zz < s.reorth * s.reorth * ww;
            s_zz = zz;
        }
    }
    __syncthreads();
    const double zz = s_second ? gm_second_pass(b, M, s.j, h2s, red) : s_zz;
    gm_commit_arnoldi(b, s, ci, h2s, sqrt(zz));
}

// The next K_D input for elements of chunk c, and with taps (the spline filter
// of a curve's density) its spline second derivatives (the filter reads
// kGmHalo neighbours on each side, wrapping around Gamma); taps is null where
// the density has no spline (the surface problem).
// Element e of the next K_D input the last commit left (kind != kGmDone): the
// updated iterate at the end of a cycle, else the normalised vector.
__device__ __forceinline__ double gm_next_x(const GmresBufs& b, int M, int kind, double scale, int jn, int e) {
    if (kind == kGmCycleEnd) {
        double x = b.phi[e];
        for (int i0 = 0; i0 < jn; i0 += 8) {
            double vv[8], yy[8];                         // the coefficients with the basis values
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const bool in = i0 + u < jn;
                vv[u] = in ? b.V[(size_t)(i0 + u) * M + e] : 0.0;
                yy[u] = in ? b.y[i0 + u] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (i0 + u < jn) x = fma(yy[u], vv[u], x);
        }
        return x;
    }
    return b.z[e] * scale;
}

// Spline second derivative at window place w (the filter reads kGmHalo places
// on each side): the same periodic filter gm_emit applies.
__device__ __forceinline__ double gm_spline_s2(const double* __restrict__ taps, const double* win, int w) {
    constexpr int K = kSplineK;
    double s = 0.0;
#pragma unroll
    for (int q = -K - 1; q <= K + 1; ++q) s = fma(taps[q + K + 1], win[w + q], s);
    return s;
}

// ctl: null in a GMRES step (everything from the state), else given by the
// launch that starts the run.
__device__ inline void gm_emit(const double* __restrict__ taps, const GmresBufs& b, int M, int c,
                               const EmitCtl* ctl = nullptr) {
    constexpr int W = kGmChunk + 2 * kGmHalo;
    __shared__ double win[W];
    const int tid = threadIdx.x, c0 = c * kGmChunk;
    // z at this thread's window places is requested before the state is read:
    // it is the next input (scaled) unless the cycle has just ended
    const double* zsrc = ctl ? ctl->xsrc : b.z;
    int ek[2];
    double zk[2];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const int k = tid + r * kGmChunk;
        int e = (c0 - kGmHalo + k) % M;
        if (e < 0) e += M;
        ek[r] = e;
        zk[r] = k < W ? zsrc[e] : 0.0;
    }
    const GmresState* st = b.st;
    const int kind = ctl ? ctl->kind : st->kind;
    if (kind == kGmDone) {                               // the run has ended: the iterate goes out
        const int e = c0 + tid;
        if (ctl) {
            if (ctl->xzero && e < M) ctl->xzero[e] = 0.0;
            return;
        }
        double* xo = st->xout;
        if (xo && st->converged != kGmNonfinite && e < M) xo[e] = b.phi[e];
        return;
    }
    const double scale = ctl ? ctl->scale : st->scale;
    const int jn = ctl ? 0 : st->jn;
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const int k = tid + r * kGmChunk;
        if (k < W) win[k] = kind == kGmCycleEnd && !ctl ? gm_next_x(b, M, kind, scale, jn, ek[r]) : zk[r] * scale;
    }
    __syncthreads();
    const int e = c0 + tid;
    if (e >= M) return;
    const double x = win[kGmHalo + tid];
    if (kind == kGmNewCycle) b.V[e] = x;
    if (kind == kGmNextVector) b.V[(size_t)st->j * M + e] = x;
    b.xcur[e] = x;
    if (!taps) return;
    b.s2cur[e] = gm_spline_s2(taps, win, kGmHalo + tid);
}

// The corrections (Alg. 2) of the next K_D apply for correction chunk cc, made
// in the same launch as gm_emit: the chunk's window of the next input is
// formed here from the same values gm_emit writes (gm_next_x), its spline
// second derivatives by the same filter, and the corrections by the same
// arithmetic as a separate correction launch after gm_emit.  One workgroup of
// kGmChunk threads; corr_il in the sparse-sum layout.
__device__ inline void gm_emit_corrections(const DevPlan& p, const GmresBufs& b, int cc, double* __restrict__ corr_il,
                                           const EmitCtl* ctl = nullptr) {
    __shared__ double xw[kCorrWindow];
    __shared__ double sw[kCorrWindow];
    const int M = p.M, tid = threadIdx.x;
    static_assert(kCorrWindow <= kGmChunk && kCorrChunk <= kGmChunk, "one window place and one node place per thread");
    // the node's plan data (place tid of the chunk's kCorrChunk) is requested
    // with the chunk itself: neither waits for the other
    int4 arm = make_int4(-1, -1, -1, -1);
    double4 dd = make_double4(0.0, 0.0, 0.0, 0.0);
    double sg = 0.0;
    int slot = 0;
    if (tid < kCorrChunk) {
        const size_t at = (size_t)cc * kCorrChunk + tid;
        arm = p.cc_arm[at];
        dd = p.cc_d[at];
        sg = p.cc_s[at];
        slot = p.cc_pos[at];
    }
    const int4 ch = p.cc_chunk[cc];                      // first, end, first knot, width
    const bool act = tid < ch.y - ch.x;
    // z at the thread's window place: the next input (scaled) unless the cycle
    // has just ended
    const int ew = (ch.z + tid) % M;
    const double zw = tid < ch.w ? (ctl ? ctl->xsrc : b.z)[ew] : 0.0;
    const int ks[4] = {arm.x, arm.y, arm.z, arm.w};
    const double ds[4] = {dd.x, dd.y, dd.z, dd.w};
    PointGeom gs[4];
    int axs[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        if (ks[a] >= 0) {
            gs[a] = p.q_geo[ks[a]];
            axs[a] = p.q_axis[ks[a]];
        } else {
            gs[a] = PointGeom{};
            axs[a] = 0;
        }
    }
    const GmresState* st = b.st;
    const int kind = ctl ? ctl->kind : st->kind;
    if (kind == kGmDone) return;
    const double scale = ctl ? ctl->scale : st->scale;
    const int jn = ctl ? 0 : st->jn;
    if (tid < ch.w) xw[tid] = kind == kGmCycleEnd && !ctl ? gm_next_x(b, M, kind, scale, jn, ew) : zw * scale;
    __syncthreads();
    for (int w = kGmHalo + tid; w < ch.w - kGmHalo; w += kGmChunk) sw[w] = gm_spline_s2(p.taps, xw, w);
    __syncthreads();
    if (!act) return;
    double acc = 0.0;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        if (ks[a] < 0) continue;
        const double d = ds[a];
        const PointGeom& g = gs[a];
        // the segment's first knot in the window; a window longer than M holds
        // some knots twice, and the copy inside the filter's reach of the
        // window's ends has no second derivative: take the other
        int l = ((g.seg - ch.z) % M + M) % M;
        if (l < kGmHalo) l += M;
        // the spline on the segment, as spline_at computes it
        const double s0 = sw[l], s1 = sw[l + 1];
        const double y0 = xw[l], y1 = xw[l + 1], u = g.u, w = 1.0 - u;
        const double sixth = 1.0 / 6.0;
        const double P = w * y0 + u * y1 + (w * w * w - w) * s0 * sixth + (u * u * u - u) * s1 * sixth;
        const double P1 = (y1 - y0) - (3.0 * w * w - 1.0) * s0 * sixth + (3.0 * u * u - 1.0) * s1 * sixth;
        const double P2 = w * s0 + u * s1;
        // the jumps, as jumps_at computes them with [F] = 0
        const double Ps = P1 * g.a1;
        double jv, gv, hh;
        if (p.normal_jump) {
            const double vtt = g.curv * P, vtn = Ps, vnn = 0.0 - vtt;
            jv = 0.0;
            if (axs[a]) {
                gv = P * g.ny;
                hh = vtt * g.ty * g.ty + 2.0 * vtn * g.ty * g.ny + vnn * g.ny * g.ny;
            } else {
                gv = P * g.nx;
                hh = vtt * g.tx * g.tx + 2.0 * vtn * g.tx * g.nx + vnn * g.nx * g.nx;
            }
        } else {
            const double Pss = P2 * g.a2 - P1 * g.a3;
            const double vtt = Pss, vtn = -g.curv * Ps, vnn = 0.0 + p.kappa * P - vtt;
            jv = P;
            if (axs[a]) {
                gv = Ps * g.ty;
                hh = vtt * g.ty * g.ty + 2.0 * vtn * g.ty * g.ny + vnn * g.ny * g.ny;
            } else {
                gv = Ps * g.tx;
                hh = vtt * g.tx * g.tx + 2.0 * vtn * g.tx * g.nx + vnn * g.nx * g.nx;
            }
        }
        acc -= sg * (jv + d * gv + 0.5 * d * d * hh);
    }
    corr_il[slot] = acc * p.inv_h2;
}

// The start of a GMRES run, one launch of kGmChunk-thread workgroups: the gc
// emit workgroups, then (with p) one per correction chunk.  Every workgroup
// first tests the initial guess phi_in (null: zero) for nonzero values and
// sums |ghat|^2 (ghat <- rhs when rhs is given, else already in place) in one
// fixed order, so all of them hold the same beta and know what the run does:
//  - a zero guess has the residual ghat itself (K 0 = 0; Alg. 5 with x_0 = 0),
//    so its first cycle starts here: V_0 = ghat / beta is the first K input;
//  - any other guess makes phi_in the first K input, and the first step is a
//    residual step;
//  - beta = 0 (x = 0 solves it) or a NaN or Inf ends the run at once.
// Workgroup 0 writes the whole state (nothing is uploaded from the host) and
// publishes it; the emit workgroups copy phi_in and rhs into phi and ghat for
// their chunk and write the first input with its spline second derivatives;
// the correction workgroups make its corrections.  xout (may be null) is where
// the emit launch of the step that ends the run copies the iterate.
__device__ inline void gm_begin(const DevPlan* p, const double* __restrict__ taps, const GmresBufs& b, int M,
                                const double* __restrict__ rhs, const double* __restrict__ phi_in, double tol,
                                int max_iter, double reorth, double* xout, double* __restrict__ corr_il) {
    __shared__ double red[kGmChunk / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, c = blockIdx.x;
    const double* gsrc = rhs ? rhs : b.ghat;
    double ss = 0.0;
    int nz = 0;
    for (int e = tid; e < M; e += kGmChunk) {
        const double gh = gsrc[e];
        if (phi_in) nz |= phi_in[e] != 0.0;               // a NaN counts as nonzero
        ss = fma(gh, gh, ss);
    }
    ss = wave_sum(ss);
    if (lane == 0) red[wave] = ss;
    const bool nonzero = __syncthreads_or(nz) != 0;
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kGmChunk / 64; ++w) t += red[w];  // fixed order
    const double beta = sqrt(t);
    EmitCtl ctl{kGmNewCycle, 1.0, gsrc, nullptr};
    int converged = 0;
    if (nonzero) {
        ctl.kind = kGmCycleEnd;
        ctl.xsrc = phi_in;
    } else if (!isfinite(beta)) {
        ctl.kind = kGmDone;
        converged = kGmNonfinite;
    } else if (beta == 0.0) {
        ctl.kind = kGmDone;
        ctl.xzero = xout;
        converged = 1;
    } else {
        ctl.scale = 1.0 / beta;
    }
    if (c == 0) {
        for (int k = 1 + tid; k <= b.m; k += kGmChunk) b.g[k] = 0.0;
        if (tid == 0) {
            GmresState* st = b.st;
            b.g[0] = nonzero ? 0.0 : beta;
            st->j = 0;
            st->it = 0;
            st->res_applies = 0;
            st->tol = tol;
            st->max_iter = max_iter;
            st->reorth = reorth;
            st->jn = 0;
            st->xout = xout;
            st->converged = converged;
            st->kind = ctl.kind;
            st->first = nonzero ? 1 : 0;
            st->r0 = nonzero ? 0.0 : beta;
            st->relres = converged == 1 ? 0.0 : 1.0;
            st->scale = ctl.scale;
            st->cycles = ctl.kind == kGmNewCycle ? 1 : 0;
            st->mode = ctl.kind == kGmNewCycle ? 1 : ctl.kind == kGmCycleEnd ? 0 : 2;
            gm_publish(b);
        }
    }
    if (c < b.gc) {
        const int e = c * kGmChunk + tid;
        if (e < M) {
            b.phi[e] = phi_in ? phi_in[e] : 0.0;
            if (rhs) b.ghat[e] = rhs[e];
        }
        gm_emit(taps, b, M, c, &ctl);
    } else {
        gm_emit_corrections(*p, b, c - b.gc, corr_il, &ctl);
    }
}

}  // namespace kfbi
