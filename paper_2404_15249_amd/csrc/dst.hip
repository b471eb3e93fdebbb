// Column sine transforms of the dense path (the fast solver's y-direction
// passes, Alg. 4 on the full grid).
//
// out[l-1][c] = alpha * sum_{j=1}^{N-1} sin(pi j l / N) in[j-1][c] (+ out[l-1][c]
// when accumulating), for every column c of an N x N row-major array whose last
// row is the zero pad of node N.  One workgroup owns B adjacent columns: it
// loads the N x B tile once (B-wide row segments), transforms it in LDS and
// writes it back in place of the same tile, so no transpose is needed.
//
// DST-I of length N-1 through one complex FFT of length N per PAIR of columns:
// with x_0 = x_N = 0 and y_j = sin(pi j/N)(x_j + x_{N-j}) + (x_j - x_{N-j})/2,
// the real DFT Y_k = R_k + i I_k of y gives X_{2k} = -I_k and
// X_{2k+1} = X_{2k-1} + R_k (X_1 = R_0/2).  Two real columns a, b are packed
// as z = y_a + i y_b and separated after the FFT by
// Y_a = (Z_k + conj Z_{N-k})/2, Y_b = -i (Z_k - conj Z_{N-k})/2.
// The FFT is an in-place radix-2 decimation-in-time transform in LDS; twiddles
// come from the quarter-period sine table.
#include <hip/hip_runtime.h>

#include "device.h"
#include "graph.h"
#include "kernels.h"

namespace kfbi {

namespace {

template <class T>
struct cpx {
    T x, y;
};

__device__ __forceinline__ int bitrev(int v, int bits) { return (int)(__brev((unsigned)v) >> (32 - bits)); }

// LDS slot of element i of a column pair's array: the low three bits of i
// XORed with a hash of the rest (a permutation inside each group of eight).
// The early FFT passes (strides 4 and 16) and the bit reversal (strides N/64
// and up) would otherwise put the lanes of a wavefront on the same banks.
__device__ __forceinline__ int zs(int i) {
    const int b = i >> 3;
    return i ^ (((b * 3) ^ ((b >> 3) * 5) ^ (b >> 6)) & 7);
}

// two adjacent columns of one row travel as one vector load or store
template <class T>
struct pair_of;
template <>
struct pair_of<double> {
    using type = double2;
};
template <>
struct pair_of<float> {
    using type = float2;
};

constexpr int kDstThreads = 1024;   // 16 wavefronts per workgroup: the LDS tile limits a CU to one
constexpr int kLoadBatch = 8;       // vector loads in flight per thread

// W_N^k = e^{-2 pi i k / N} for 0 <= k < N, from the quarter-period table
__device__ __forceinline__ void twiddle(const double* sq, int k, int N, double& wr, double& wi) {
    const int mask2 = 2 * N - 1;
    wr = sinpi_n(sq, (2 * k + N / 2) & mask2, N);
    wi = -sinpi_n(sq, (2 * k) & mask2, N);
}

// Passes s and s+1 of the decimation-in-time FFT on four points at distance h
// (a radix-4 step): with k = pos N / (4h) the table gives W = W_N^k; pass s
// combines (a, b) and (c, d) with W^2, pass s+1 combines (a, c) with W and
// (b, d) with W_N^{k + N/4} = -i W.  In place.
template <class T>
__device__ __forceinline__ void radix4_step(const double* sq, int tw, int N, cpx<T>& a, cpx<T>& bb, cpx<T>& c,
                                            cpx<T>& d) {
    double dr, di;
    twiddle(sq, tw, N, dr, di);
    const T w2r = (T)dr, w2i = (T)di;
    const T w1r = (T)(dr * dr - di * di), w1i = (T)(2.0 * dr * di);
    // pass s: (a, b) and (c, d) with W^2
    const T tbr = w1r * bb.x - w1i * bb.y, tbi = w1r * bb.y + w1i * bb.x;
    const T tdr = w1r * d.x - w1i * d.y, tdi = w1r * d.y + w1i * d.x;
    const cpx<T> a1{a.x + tbr, a.y + tbi}, b1{a.x - tbr, a.y - tbi};
    const cpx<T> c1{c.x + tdr, c.y + tdi}, d1{c.x - tdr, c.y - tdi};
    // pass s + 1: (a, c) with W and (b, d) with -i W
    const T tcr = w2r * c1.x - w2i * c1.y, tci = w2r * c1.y + w2i * c1.x;
    const T ter = w2i * d1.x + w2r * d1.y, tei = w2i * d1.y - w2r * d1.x;
    a = cpx<T>{a1.x + tcr, a1.y + tci};
    c = cpx<T>{a1.x - tcr, a1.y - tci};
    bb = cpx<T>{b1.x + ter, b1.y + tei};
    d = cpx<T>{b1.x - ter, b1.y - tei};
}

// Rows are ld elements apart; blockIdx.y selects a slice of `slice` elements
// (several independent N-row arrays, as the planes of a 3D grid).
template <class T, class Tin, class Tout, int B>
__global__ __launch_bounds__(kDstThreads) void k_dst_cols(int N, int log2N, const double* __restrict__ sinq,
                                                          const Tin* in, Tout* out, double alpha, int accumulate,
                                                          int ld, size_t slice, const int* __restrict__ skip) {
    if (skip && *skip) return;
    in += blockIdx.y * slice;
    out += blockIdx.y * slice;
    extern __shared__ double smem_d[];
    constexpr int P = B / 2;                                 // column pairs
    constexpr int LP = B == 4 ? 1 : B == 8 ? 2 : 3;          // log2 P
    constexpr int NTH = kDstThreads;
    using Vin = typename pair_of<Tin>::type;
    using Vout = typename pair_of<Tout>::type;
    const int NS = N + 1;                                    // pair stride (one pad entry)
    double* sq = smem_d;                                     // N/2 + 2
    cpx<T>* z = reinterpret_cast<cpx<T>*>(smem_d + (N / 2 + 2));   // P x NS
    const int tid = threadIdx.x;
    // XCD-aware tile order: consecutive workgroups go round-robin over the 8
    // XCDs, so give each XCD a contiguous range of tiles; neighbouring tiles
    // share the cache lines of their row segments in that XCD's L2
    const int G = gridDim.x;
    const int tile = (G & 7) ? (int)blockIdx.x : ((int)blockIdx.x & 7) * (G >> 3) + ((int)blockIdx.x >> 3);
    const int col0 = tile * B;
    for (int k = tid; k <= N / 2; k += NTH) sq[k] = sinq[k];
    // load and pre-process in one pass: item (j, p), j = 1 .. N/2, loads x_j
    // (row j-1) and x_{N-j} (row N-j-1) of column pair p, forms y_j and y_{N-j}
    // and stores them at their bit-reversed places, the order the
    // decimation-in-time passes read (so no reversal pass); x_0 = x_N = 0 gives
    // y_0 = 0.  A batch's loads are all issued before any is used.
    const int lh = log2N - 1;                                // log2 (N/2)
    constexpr int LB = kLoadBatch / 2;
    const int items = P << lh;
    for (int base = 0; base < items; base += NTH * LB) {
        Vin va[LB], vb[LB];
        double sv[LB];
#pragma unroll
        for (int u = 0; u < LB; ++u) {
            const int idx = base + u * NTH + tid;
            const int j = (idx >> LP) + 1, p = idx & (P - 1);
            if (idx < items) {
                va[u] = *reinterpret_cast<const Vin*>(in + (size_t)(j - 1) * ld + col0 + 2 * p);
                if (j < N / 2) vb[u] = *reinterpret_cast<const Vin*>(in + (size_t)(N - j - 1) * ld + col0 + 2 * p);
                sv[u] = sinq[j];
            }
        }
#pragma unroll
        for (int u = 0; u < LB; ++u) {
            const int idx = base + u * NTH + tid;
            const int j = (idx >> LP) + 1, p = idx & (P - 1);
            if (idx >= items) continue;
            cpx<T>* zp = z + p * NS;
            const T ax = (T)va[u].x, ay = (T)va[u].y;
            if (j == N / 2) {
                zp[zs(bitrev(j, log2N))] = cpx<T>{ax * T(2), ay * T(2)};
            } else {
                const T bx = (T)vb[u].x, by = (T)vb[u].y;
                const T sj = (T)sv[u];
                zp[zs(bitrev(j, log2N))] = cpx<T>{sj * (ax + bx) + T(0.5) * (ax - bx), sj * (ay + by) + T(0.5) * (ay - by)};
                zp[zs(bitrev(N - j, log2N))] =
                    cpx<T>{sj * (bx + ax) + T(0.5) * (bx - ax), sj * (by + ay) + T(0.5) * (by - ay)};
            }
        }
    }
    if (tid < P) z[tid * NS + zs(0)] = cpx<T>{T(0), T(0)};
    __syncthreads();
    // passes s .. s+3 together as one radix-16 step (h = 2^(s-1), 16 points
    // at distance h held in registers): two radix-4 steps, the first on the
    // four groups of four consecutive points (passes s, s+1: one twiddle for
    // all four), the second across the groups (passes s+2, s+3: distance 4h,
    // the twiddle of each point's own position); one LDS round trip for four
    // passes.  Then radix-4 steps (passes s, s+1) while two passes are left.
    int s = 1;
    const int lx = log2N - 4;                                // log2 (N/16)
    for (; s + 3 <= log2N; s += 4) {
        const int h = 1 << (s - 1);
        for (int idx = tid; idx < (P << lx); idx += NTH) {
            const int p = idx >> lx, b = idx & (N / 16 - 1);
            const int pos = b & (h - 1), grp = b >> (s - 1);
            const int i0 = grp * 16 * h + pos;
            cpx<T>* zp = z + p * NS;
            cpx<T> x[16];
#pragma unroll
            for (int q = 0; q < 16; ++q) x[q] = zp[zs(i0 + q * h)];
            const int tw1 = pos << (log2N - s - 1);
#pragma unroll
            for (int t = 0; t < 4; ++t) radix4_step(sq, tw1, N, x[4 * t], x[4 * t + 1], x[4 * t + 2], x[4 * t + 3]);
#pragma unroll
            for (int q = 0; q < 4; ++q)
                radix4_step(sq, (pos + q * h) << (log2N - s - 3), N, x[q], x[q + 4], x[q + 8], x[q + 12]);
#pragma unroll
            for (int q = 0; q < 16; ++q) zp[zs(i0 + q * h)] = x[q];
        }
        __syncthreads();
    }
    const int lq = log2N - 2;                                // log2 (N/4)
    for (; s + 1 <= log2N; s += 2) {
        const int h = 1 << (s - 1);
        for (int idx = tid; idx < (P << lq); idx += NTH) {
            const int p = idx >> lq, b = idx & (N / 4 - 1);
            const int pos = b & (h - 1), grp = b >> (s - 1);
            const int i0 = grp * 4 * h + pos;
            cpx<T>* zp = z + p * NS;
            cpx<T> a = zp[zs(i0)], bb = zp[zs(i0 + h)], c = zp[zs(i0 + 2 * h)], d = zp[zs(i0 + 3 * h)];
            radix4_step(sq, pos << (log2N - s - 1), N, a, bb, c, d);
            zp[zs(i0)] = a;
            zp[zs(i0 + h)] = bb;
            zp[zs(i0 + 2 * h)] = c;
            zp[zs(i0 + 3 * h)] = d;
        }
        __syncthreads();
    }
    if (s == log2N) {                                        // odd log2 N: one radix-2 pass left
        const int half = 1 << (s - 1);
        for (int idx = tid; idx < (P << lh); idx += NTH) {
            const int p = idx >> lh, pos = idx & (N / 2 - 1);
            const int i1 = pos, i2 = pos + half;
            double dr, di;
            twiddle(sq, pos, N, dr, di);
            const T wr = (T)dr, wi = (T)di;
            cpx<T>* zp = z + p * NS;
            const cpx<T> a = zp[zs(i1)], c = zp[zs(i2)];
            const T tr = wr * c.x - wi * c.y, ti = wr * c.y + wi * c.x;
            zp[zs(i1)] = cpx<T>{a.x + tr, a.y + ti};
            zp[zs(i2)] = cpx<T>{a.x - tr, a.y - ti};
        }
        __syncthreads();
    }
    // separate the two columns: slot k <- (R_a, R_b), slot N-k <- (-I_a, -I_b) = X_2k
    for (int idx = tid; idx < (P << lh); idx += NTH) {
        const int p = idx >> lh, k = idx & (N / 2 - 1);
        cpx<T>* zp = z + p * NS;
        const cpx<T> Zk = zp[zs(k)], Zn = zp[zs((N - k) & (N - 1))];
        const T ra = T(0.5) * (Zk.x + Zn.x), ia = T(0.5) * (Zk.y - Zn.y);
        const T rb = T(0.5) * (Zk.y + Zn.y), ib = -T(0.5) * (Zk.x - Zn.x);
        zp[zs(k)] = cpx<T>{ra, rb};
        if (k > 0) zp[zs(N - k)] = cpx<T>{-ia, -ib};
    }
    __syncthreads();
    // odd outputs: X_{2k+1} = R_0/2 + R_1 + ... + R_k, one wavefront per column.
    // Lane t owns the L values t L .. t L + L - 1 and visits them rotated by
    // t mod L, so that the lanes of a wavefront read different LDS banks; the
    // values before the rotation point are summed separately, which keeps
    // every running sum in index order.  Running sums are carried in FP64
    // whatever the storage type.
    if (tid < 64 * B) {
        const int c = tid >> 6, t = tid & 63;
        const int tpc = min(64, N / 2);                      // lanes with values
        const int lL = (log2N - 1) - (tpc == 64 ? 6 : log2N - 1);
        const int L = 1 << lL;
        const int off = t & (L - 1);
        T* col = reinterpret_cast<T*>(z + (c >> 1) * NS) + (c & 1);   // element k at col[2 k]
        double lo = 0.0, hi = 0.0;                           // values before / from the rotation point
        if (t < tpc) {
            for (int q = 0; q < L; ++q) {
                const int e = (q + off) & (L - 1), k = (t << lL) + e;
                double v = (double)col[2 * zs(k)];
                if (k == 0) v *= 0.5;
                if (e >= off) hi += v; else lo += v;
            }
        }
        double incl = lo + hi;
        for (int o = 1; o < 64; o <<= 1) {
            const double u = __shfl_up(incl, o, 64);
            if (t >= o) incl += u;
        }
        double excl = __shfl_up(incl, 1, 64);
        if (t == 0) excl = 0.0;
        if (t < tpc) {
            double acc_hi = excl + lo, acc_lo = excl;
            for (int q = 0; q < L; ++q) {
                const int e = (q + off) & (L - 1), k = (t << lL) + e;
                double v = (double)col[2 * zs(k)];
                if (k == 0) v *= 0.5;
                double w;
                if (e >= off) w = (acc_hi += v); else w = (acc_lo += v);
                col[2 * zs(k)] = (T)w;
            }
        }
    }
    __syncthreads();
    // write: X_l to row l-1 (odd l from slot (l-1)/2, even l from slot N - l/2); row N-1 is the pad
    for (int base = 0; base < N * P; base += NTH * kLoadBatch) {
        double vx[kLoadBatch], vy[kLoadBatch];
#pragma unroll
        for (int u = 0; u < kLoadBatch; ++u) {
            const int idx = base + u * NTH + tid;
            const int r = idx >> LP, p = idx & (P - 1);
            const int l = r + 1;
            vx[u] = vy[u] = 0.0;
            if (idx < N * P && l < N) {
                const cpx<T> e = z[p * NS + zs((l & 1) ? (l - 1) >> 1 : N - (l >> 1))];
                vx[u] = alpha * (double)e.x;
                vy[u] = alpha * (double)e.y;
            }
        }
        if (accumulate) {
            Vout old[kLoadBatch];
#pragma unroll
            for (int u = 0; u < kLoadBatch; ++u) {
                const int idx = base + u * NTH + tid;
                const int r = idx >> LP, p = idx & (P - 1);
                if (idx < N * P) old[u] = *reinterpret_cast<const Vout*>(out + (size_t)r * ld + col0 + 2 * p);
            }
#pragma unroll
            for (int u = 0; u < kLoadBatch; ++u) {
                vx[u] += (double)old[u].x;
                vy[u] += (double)old[u].y;
            }
        }
#pragma unroll
        for (int u = 0; u < kLoadBatch; ++u) {
            const int idx = base + u * NTH + tid;
            const int r = idx >> LP, p = idx & (P - 1);
            Vout o;
            o.x = (Tout)vx[u];
            o.y = (Tout)vy[u];
            if (idx < N * P) *reinterpret_cast<Vout*>(out + (size_t)r * ld + col0 + 2 * p) = o;
        }
    }
}

// The transform geometry of one launch: N-row arrays with rows ld elements
// apart and ld columns, `slices` of them `slice` elements apart.
struct Lines {
    int N, log2N;
    const double* sinq;
    int ld, slices;
    size_t slice;
    const int* skip;
};

template <class T, class Tin, class Tout, int B>
hipError_t dst_launch(const Lines& g, const Tin* in, Tout* out, double alpha, bool acc, hipStream_t s) {
    const size_t lds = dst_lds_bytes(g.N, B, sizeof(cpx<T>));
    if (hipError_t e = hipFuncSetAttribute((const void*)k_dst_cols<T, Tin, Tout, B>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds))
        return e;
    if (hipError_t e_ = klaunch(&k_dst_cols<T, Tin, Tout, B>, dim3(g.ld / B, g.slices), dim3(kDstThreads), lds, s,
                                g.N, g.log2N, g.sinq, in, out, alpha, acc ? 1 : 0, g.ld, g.slice, g.skip))
        return e_;
    return hipGetLastError();
}

template <class T, class Tin, class Tout>
hipError_t dst_dispatch(const Lines& g, const Tin* in, Tout* out, double alpha, bool acc, int B, hipStream_t s) {
    if (!dst_tile_ok(g.N, B, sizeof(cpx<T>), ~(size_t)0) || g.ld % B != 0) return hipErrorInvalidValue;
    switch (B) {
        case 4: return dst_launch<T, Tin, Tout, 4>(g, in, out, alpha, acc, s);
        case 8: return dst_launch<T, Tin, Tout, 8>(g, in, out, alpha, acc, s);
        default: return dst_launch<T, Tin, Tout, 16>(g, in, out, alpha, acc, s);
    }
}

Lines grid2(const DevPlan& p) { return Lines{p.N, p.log2N, p.sinq, p.N, 1, 0, nullptr}; }

}  // namespace

size_t dst_lds_bytes(int N, int B, size_t cpx_bytes) {
    return sizeof(double) * (size_t)(N / 2 + 2) + cpx_bytes * (size_t)(B / 2) * (N + 1);
}

bool dst_tile_ok(int N, int B, size_t cpx_bytes, size_t lds_max) {
    // 256 / B threads per column share a scan of N / 2 values with wavefront shuffles
    if (B != 4 && B != 8 && B != 16) return false;
    if (N % B || 256 / B > 64 || (N / 2) < 256 / B) return false;
    return dst_lds_bytes(N, B, cpx_bytes) <= lds_max;
}

int dst_default_tile(int N, size_t cpx_bytes, size_t lds_max, long lines, int min_groups) {
    // the widest valid tile that still gives min_groups workgroups (wider
    // tiles read longer row segments, more workgroups fill the chip); else the
    // narrowest valid one
    for (int B : {16, 8, 4})
        if (dst_tile_ok(N, B, cpx_bytes, lds_max) && lines / B >= min_groups) return B;
    for (int B : {4, 8, 16})
        if (dst_tile_ok(N, B, cpx_bytes, lds_max)) return B;
    return 0;
}

hipError_t launch_dst_cols(const DevPlan& p, const double* in, double* out, double alpha, bool acc, int B,
                           hipStream_t s) {
    return dst_dispatch<double>(grid2(p), in, out, alpha, acc, B, s);
}

hipError_t launch_dst_cols_f32(const DevPlan& p, const double* in, float* out, double alpha, int B, hipStream_t s) {
    return dst_dispatch<float>(grid2(p), in, out, alpha, false, B, s);
}

hipError_t launch_dst_cols_f32_to64(const DevPlan& p, const float* in, double* out, double alpha, bool acc, int B,
                                    hipStream_t s) {
    return dst_dispatch<float>(grid2(p), in, out, alpha, acc, B, s);
}

hipError_t launch_dst_lines(int N, int log2N, const double* sinq, double* a, double alpha, int B, int ld, int slices,
                            size_t slice, const int* skip, hipStream_t s) {
    return dst_dispatch<double>(Lines{N, log2N, sinq, ld, slices, slice, skip}, a, a, alpha, false, B, s);
}

}  // namespace kfbi
