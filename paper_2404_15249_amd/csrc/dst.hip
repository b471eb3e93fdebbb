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

#include <algorithm>

#include "device.h"
#include "graph.h"
#include "kernels.h"

namespace kfbi {

namespace {

// aligned to its size, so that one element moves as one 16-byte (8-byte) LDS
// access: the bank rules below assume that width
template <class T>
struct alignas(2 * sizeof(T)) cpx {
    T x, y;
};

// a compile-time int passed as an argument (selects a generic lambda's body)
template <int V>
struct IntConst {
    static constexpr int value = V;
};

__device__ __forceinline__ int bitrev(int v, int bits) { return (int)(__brev((unsigned)v) >> (32 - bits)); }

// LDS banks on gfx950: 64 four-byte banks.  A 16-byte access serves the
// lanes of a wavefront in four groups of 16 (lanes 0-3, 12-15, 20-27 and
// 4-11, 16-19, 28-31, the same in the upper half), an 8-byte access in two
// groups of 32 (the half-waves); an access takes one pass per group when the
// group's lanes fall on distinct 16-byte (8-byte) slots of a 256-byte row.
// Every group holds one lane of each residue mod 16, so consecutive elements
// across a group never clash.
//
// LDS slot of element i of a column pair's array: a permutation inside each
// aligned block of 16 (16-byte pairs) or 32 (8-byte pairs) that XORs the low
// bits with higher ones.  A radix pass at stride h reads i0 + q h with
// consecutive lanes on consecutive i0 for h >= 16 and on consecutive
// (i0 >> 4) for h = 1; the XOR spreads both over a bank row.  16-byte pairs:
// bits 4-7 into bits 0-3.
template <class T>
__device__ __forceinline__ int zs(int i) {
    if constexpr (sizeof(T) == 8) return i ^ ((i >> 4) & 15);
    // 8-byte pairs, 32 lanes a pass: bits 5-8 into bits 0-3 (stride 1 and
    // stride-16 passes) and bit 8 into bit 4 (the stride-16 pass's lanes
    // differ in bits 0-3 and 8)
    return i ^ ((i >> 5) & 15) ^ (((i >> 8) & 1) << 4);
}

// Slot of element i of pair p.  With 8 or more pairs (16-byte pairs only) a
// wavefront of the early passes spans several pairs, so the pair index joins
// the XOR: lanes of different pairs with the same element land apart.
template <class T, int P>
__device__ __forceinline__ int zsp(int p, int i) {
    if constexpr (sizeof(T) == 8 && P >= 8) return i ^ (((i >> 4) ^ p) & 15);
    return zs<T>(i);
}

// Slot of point i0 + q h of pair p in a pass at stride h, from a = its slot for
// q = 0.  The passes run at h = 1, 16 or a multiple of 256 with i0 free of the
// bits of q h, so i0 + q h = i0 ^ q h, and the 16-byte pairs' swizzle then moves
// the slot by q h, plus q when h = 16 (bits 4-7 of the element index change with
// q).  One XOR per point instead of the swizzle's arithmetic.
template <class T, int P>
__device__ __forceinline__ int pass_slot(int a, int p, int i0, int q, int h) {
    if constexpr (sizeof(T) == 8) return a ^ (q * h) ^ (h == 16 ? q : 0);
    return zsp<T, P>(p, i0 + q * h);
}

// pair stride N + pad: the load and write phases interleave the P pairs
// across lanes, so successive pairs start a 1/P bank row apart (with 8 or
// more pairs the XOR above spreads them instead)
template <class T, int B>
constexpr int pair_pad() {
    constexpr int P = B / 2;
    if constexpr (sizeof(T) == 8) return P <= 4 ? 16 / P : P == 8 ? 8 : 0;
    return 32 / P;
}

// The twiddle table: W_N^k = (cos 2 pi k/N, -sin 2 pi k/N) for 0 <= k < N/4, one
// 16-byte entry each, entry k at slot k ^ ((k >> 4 ^ k >> 8) & 15) (a
// permutation inside each aligned block of 16) so that the reads of every pass
// at its power-of-two strides land on distinct banks.
__device__ __forceinline__ int tws(int k) { return k ^ (((k >> 4) ^ (k >> 8)) & 15); }

// doubles of LDS the table takes (N/4 pairs); the pair arrays follow it
__host__ __device__ constexpr int dst_table_len(int N) { return N / 2; }

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

// W_N^k for 0 <= k < N/2 from the table: W_N^{k + N/4} = -i W_N^k
__device__ __forceinline__ void twiddle(const cpx<double>* tw, int k, int N, double& wr, double& wi) {
    const int q = N / 4;
    const cpx<double> w = tw[tws(k & (q - 1))];
    if (k & q) {
        wr = w.y;
        wi = -w.x;
    } else {
        wr = w.x;
        wi = w.y;
    }
}

// Passes s and s+1 of the decimation-in-time FFT on four points at distance h
// (a radix-4 step): with k = pos N / (4h) the table gives W = W_N^k; pass s
// combines (a, b) and (c, d) with W^2, pass s+1 combines (a, c) with W and
// (b, d) with W_N^{k + N/4} = -i W.  In place.
template <class T>
__device__ __forceinline__ void radix4_step(double dr, double di, cpx<T>& a, cpx<T>& bb, cpx<T>& c, cpx<T>& d) {
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

// the same with the twiddle read from the table
template <class T>
__device__ __forceinline__ void radix4_step(const cpx<double>* sq, int tw, int N, cpx<T>& a, cpx<T>& bb, cpx<T>& c,
                                            cpx<T>& d) {
    double dr, di;
    twiddle(sq, tw, N, dr, di);
    radix4_step(dr, di, a, bb, c, d);
}

// The radix-4 step with W = 1 (the first passes, h = 1): additions only
// (pass s + 1 multiplies (b, d) by -i)
template <class T>
__device__ __forceinline__ void radix4_unit(cpx<T>& a, cpx<T>& bb, cpx<T>& c, cpx<T>& d) {
    const cpx<T> a1{a.x + bb.x, a.y + bb.y}, b1{a.x - bb.x, a.y - bb.y};
    const cpx<T> c1{c.x + d.x, c.y + d.y}, d1{c.x - d.x, c.y - d.y};
    a = cpx<T>{a1.x + c1.x, a1.y + c1.y};
    c = cpx<T>{a1.x - c1.x, a1.y - c1.y};
    bb = cpx<T>{b1.x + d1.y, b1.y - d1.x};
    d = cpx<T>{b1.x - d1.y, b1.y + d1.x};
}

// Inclusive sums over aligned groups of W consecutive lanes (W = 16, 32 or
// 64): four DPP row shifts inside each row of 16 lanes, then the row totals
// read as scalars and added in row order.
__device__ __forceinline__ double group_scan(double v, int W, int lane) {
    v += dpp_f64<kDppRowShr1>(v);
    v += dpp_f64<kDppRowShr1 + 1>(v);
    v += dpp_f64<kDppRowShr1 + 3>(v);
    v += dpp_f64<kDppRowShr1 + 7>(v);
    if (W > 16) {
        const double r0 = readlane_f64(v, 15), r1 = readlane_f64(v, 31), r2 = readlane_f64(v, 47);
        const int row = lane >> 4;
        double before;
        if (W == 32)
            before = row == 1 ? r0 : row == 3 ? r2 : 0.0;
        else
            before = row == 1 ? r0 : row == 2 ? r0 + r1 : row == 3 ? (r0 + r1) + r2 : 0.0;
        v += before;
    }
    return v;
}

// Pass s' on two points at distance 2^(s'-1): b <- a - W b, a <- a + W b with
// W = W_N^tw.  In place.
template <class T>
__device__ __forceinline__ void radix2_step(double dr, double di, cpx<T>& a, cpx<T>& b) {
    const T wr = (T)dr, wi = (T)di;
    const T tr = wr * b.x - wi * b.y, ti = wr * b.y + wi * b.x;
    b = cpx<T>{a.x - tr, a.y - ti};
    a = cpx<T>{a.x + tr, a.y + ti};
}

template <class T>
__device__ __forceinline__ void radix2_step(const cpx<double>* sq, int tw, int N, cpx<T>& a, cpx<T>& b) {
    double dr, di;
    twiddle(sq, tw, N, dr, di);
    radix2_step(dr, di, a, b);
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
    constexpr int LP = B == 4 ? 1 : B == 8 ? 2 : B == 16 ? 3 : B == 32 ? 4 : 5;   // log2 P
    constexpr int NTH = kDstThreads;
    using Vin = typename pair_of<Tin>::type;
    using Vout = typename pair_of<Tout>::type;
    const int NS = N + pair_pad<T, B>();                     // pair stride
    cpx<double>* sq = reinterpret_cast<cpx<double>*>(smem_d);   // twiddle table
    cpx<T>* z = reinterpret_cast<cpx<T>*>(smem_d + dst_table_len(N));   // P x NS
    const int tid = threadIdx.x;
    // XCD-aware tile order: consecutive workgroups go round-robin over the 8
    // XCDs, so give each XCD a contiguous range of tiles; neighbouring tiles
    // share the cache lines of their row segments in that XCD's L2
    const int G = gridDim.x;
    const int tile = (G & 7) ? (int)blockIdx.x : ((int)blockIdx.x & 7) * (G >> 3) + ((int)blockIdx.x >> 3);
    const int col0 = tile * B;
    for (int k = tid; k < N / 4; k += NTH) sq[tws(k)] = cpx<double>{sinq[N / 2 - 2 * k], -sinq[2 * k]};
    // load and pre-process in one pass.  With rev the log2 N-bit reversal, the
    // passes read y_j at place rev(j); y_j and y_{N-j} need x_j (row j-1) and
    // x_{N-j} (row N-j-1).  Item q = 0 .. N/2-1 of column pair p takes the
    // place i = 2 lo - r (r = N/2 - q, lo the power of two >= r) and its
    // partner i ^ (lo - 1), whose reversal is N - rev(i): the places of each
    // power-of-two range [lo, 2 lo) pair its first half with its second half
    // reversed, so the items meet every pair {j, N - j} once (i = 1 is
    // j = N/2, its own partner) and a wavefront's stores run through
    // consecutive places, ascending and descending.  x_0 = x_N = 0 gives
    // y_0 = 0.  A batch's loads are all issued before any is used, and every
    // path uses every loaded value (no load is left outstanding into the
    // next batch, so the compiler need not wait between one item's loads and
    // the next's): i = 1 (j = N/2) reads its one row twice and the table's
    // sin(pi/2) = 1, which gives 2 x_j through the general formula, stored at
    // place 1 twice; threads past the last item redo it (the same values to
    // the same places).
    const int lh = log2N - 1;                                // log2 (N/2)
    constexpr int LB = kLoadBatch / 2;
    const int items = P << lh;
    auto place = [&](int q, int& lo) {
        const int r = N / 2 - q;                             // 1 .. N/2
        lo = r <= 1 ? 1 : 1 << (32 - __clz(r - 1));
        return 2 * lo - r;
    };
    for (int base = 0; base < items; base += NTH * LB) {
        Vin va[LB], vb[LB];
        double sv[LB];
#pragma unroll
        for (int u = 0; u < LB; ++u) {
            const int idx = min(base + u * NTH + tid, items - 1);
            const int p = idx & (P - 1);
            int lo;
            const int i = place(idx >> LP, lo);
            const int j = bitrev(i, log2N);
            va[u] = *reinterpret_cast<const Vin*>(in + (size_t)(j - 1) * ld + col0 + 2 * p);
            vb[u] = *reinterpret_cast<const Vin*>(in + (size_t)(N - j - 1) * ld + col0 + 2 * p);
            sv[u] = sinq[min(j, N - j)];
        }
#pragma unroll
        for (int u = 0; u < LB; ++u) {
            const int idx = min(base + u * NTH + tid, items - 1);
            const int p = idx & (P - 1);
            int lo;
            const int i = place(idx >> LP, lo);
            cpx<T>* zp = z + p * NS;
            const T ax = (T)va[u].x, ay = (T)va[u].y;
            const T bx = (T)vb[u].x, by = (T)vb[u].y;
            const T sj = (T)sv[u];
            zp[zsp<T, P>(p, i)] = cpx<T>{sj * (ax + bx) + T(0.5) * (ax - bx), sj * (ay + by) + T(0.5) * (ay - by)};
            zp[zsp<T, P>(p, i ^ (lo - 1))] =
                cpx<T>{sj * (bx + ax) + T(0.5) * (bx - ax), sj * (by + ay) + T(0.5) * (by - ay)};
        }
    }
    if (tid < P) z[tid * NS + zsp<T, P>(tid, 0)] = cpx<T>{T(0), T(0)};
    __syncthreads();
    // passes s .. s+3 together as one radix-16 step (h = 2^(s-1), 16 points
    // at distance h held in registers): two radix-4 steps, the first on the
    // four groups of four consecutive points (passes s, s+1: one twiddle for
    // all four), the second across the groups (passes s+2, s+3: distance 4h,
    // the twiddle of each point's own position); one LDS round trip for four
    // passes.  What is left after them: three passes as one radix-8 step, else
    // radix-4 steps and a last radix-2 pass.
    const int lx = log2N - 4;                                // log2 (N/16)
    // passes 1 .. 4 (h = 1, N >= 32 always has them): the first radix-4
    // steps' twiddle is W^0 = 1, so they are additions only; the second
    // stage's are W_N^{q N/16}, the same for every item
    {
        for (int idx = tid; idx < (P << lx); idx += NTH) {
            const int p = idx >> lx, i0 = (idx & (N / 16 - 1)) * 16;
            cpx<T>* zp = z + p * NS;
            cpx<T> x[16];
            const int a0 = zsp<T, P>(p, i0);
#pragma unroll
            for (int q = 0; q < 16; ++q) x[q] = zp[pass_slot<T, P>(a0, p, i0, q, 1)];
#pragma unroll
            for (int t = 0; t < 4; ++t) radix4_unit(x[4 * t], x[4 * t + 1], x[4 * t + 2], x[4 * t + 3]);
#pragma unroll
            for (int q = 0; q < 4; ++q) radix4_step(sq, q << lx, N, x[q], x[q + 4], x[q + 8], x[q + 12]);
#pragma unroll
            for (int q = 0; q < 16; ++q) zp[pass_slot<T, P>(a0, p, i0, q, 1)] = x[q];
        }
        __syncthreads();
    }
    int s = 5;
    for (; s + 3 <= log2N; s += 4) {
        const int h = 1 << (s - 1);
        for (int idx = tid; idx < (P << lx); idx += NTH) {
            const int p = idx >> lx, b = idx & (N / 16 - 1);
            const int pos = b & (h - 1), grp = b >> (s - 1);
            const int i0 = grp * 16 * h + pos;
            cpx<T>* zp = z + p * NS;
            cpx<T> x[16];
            const int a0 = zsp<T, P>(p, i0);
#pragma unroll
            for (int q = 0; q < 16; ++q) x[q] = zp[pass_slot<T, P>(a0, p, i0, q, h)];
            // the five twiddles are read before any is used
            double w1r, w1i, w2r[4], w2i[4];
            twiddle(sq, pos << (log2N - s - 1), N, w1r, w1i);
#pragma unroll
            for (int q = 0; q < 4; ++q) twiddle(sq, (pos + q * h) << (log2N - s - 3), N, w2r[q], w2i[q]);
#pragma unroll
            for (int t = 0; t < 4; ++t) radix4_step(w1r, w1i, x[4 * t], x[4 * t + 1], x[4 * t + 2], x[4 * t + 3]);
#pragma unroll
            for (int q = 0; q < 4; ++q) radix4_step(w2r[q], w2i[q], x[q], x[q + 4], x[q + 8], x[q + 12]);
#pragma unroll
            for (int q = 0; q < 16; ++q) zp[pass_slot<T, P>(a0, p, i0, q, h)] = x[q];
        }
        __syncthreads();
    }
    // three passes left: one radix-8 step (a radix-4 step on each half, then
    // pass s+2 at distance 4h, twiddle W_N^{(pos + q h) N / (8h)} for point q)
    if (s + 2 == log2N) {
        const int h = 1 << (s - 1);
        const int l8 = log2N - 3;                            // log2 (N/8)
        for (int idx = tid; idx < (P << l8); idx += NTH) {
            const int p = idx >> l8, b = idx & (N / 8 - 1);
            const int pos = b & (h - 1), grp = b >> (s - 1);
            const int i0 = grp * 8 * h + pos;
            cpx<T>* zp = z + p * NS;
            cpx<T> x[8];
            const int a0 = zsp<T, P>(p, i0);
#pragma unroll
            for (int q = 0; q < 8; ++q) x[q] = zp[pass_slot<T, P>(a0, p, i0, q, h)];
            // the five twiddles are read before any is used
            double w1r, w1i, w2r[4], w2i[4];
            twiddle(sq, pos << (log2N - s - 1), N, w1r, w1i);
#pragma unroll
            for (int q = 0; q < 4; ++q) twiddle(sq, (pos + q * h) << (log2N - s - 2), N, w2r[q], w2i[q]);
            radix4_step(w1r, w1i, x[0], x[1], x[2], x[3]);
            radix4_step(w1r, w1i, x[4], x[5], x[6], x[7]);
#pragma unroll
            for (int q = 0; q < 4; ++q) radix2_step(w2r[q], w2i[q], x[q], x[q + 4]);
#pragma unroll
            for (int q = 0; q < 8; ++q) zp[pass_slot<T, P>(a0, p, i0, q, h)] = x[q];
        }
        __syncthreads();
        s += 3;
    }
    const int lq = log2N - 2;                                // log2 (N/4)
    for (; s + 1 <= log2N; s += 2) {
        const int h = 1 << (s - 1);
        for (int idx = tid; idx < (P << lq); idx += NTH) {
            const int p = idx >> lq, b = idx & (N / 4 - 1);
            const int pos = b & (h - 1), grp = b >> (s - 1);
            const int i0 = grp * 4 * h + pos;
            cpx<T>* zp = z + p * NS;
            const int a0 = zsp<T, P>(p, i0);
            const int s1 = pass_slot<T, P>(a0, p, i0, 1, h), s2 = pass_slot<T, P>(a0, p, i0, 2, h),
                      s3 = pass_slot<T, P>(a0, p, i0, 3, h);
            cpx<T> a = zp[a0], bb = zp[s1], c = zp[s2], d = zp[s3];
            radix4_step(sq, pos << (log2N - s - 1), N, a, bb, c, d);
            zp[a0] = a;
            zp[s1] = bb;
            zp[s2] = c;
            zp[s3] = d;
        }
        __syncthreads();
    }
    if (s == log2N) {                                        // one radix-2 pass left
        const int half = 1 << (s - 1);
        for (int idx = tid; idx < (P << lh); idx += NTH) {
            const int p = idx >> lh, pos = idx & (N / 2 - 1);
            cpx<T>* zp = z + p * NS;
            const int a0 = zsp<T, P>(p, pos), s1 = pass_slot<T, P>(a0, p, pos, 1, half);
            cpx<T> a = zp[a0], c = zp[s1];
            radix2_step(sq, pos, N, a, c);
            zp[a0] = a;
            zp[s1] = c;
        }
        __syncthreads();
    }
    // separate the two columns and sum the odd outputs.  From Z_k and
    // Z_{N-k}: (R_a, R_b) = (Re, Im) of (Z_k + conj Z_{N-k}) / 2 and
    // (I_a, I_b) = (Im, -Re) of (Z_k - conj Z_{N-k}) / 2; X_{2k} = -I_k goes
    // to slot N-k at once (only the thread owning k reads that slot), and
    // X_{2k+1} = R_0/2 + R_1 + ... + R_k to slot k.  TPP threads per pair own
    // V consecutive k each: a running sum over the thread's values, an
    // inclusive scan of the thread totals across the wavefront (DPP), then the
    // totals of the pair's earlier wavefronts, added in wavefront order
    // (through LDS, in the place of the sine table, which is no longer read).
    // Sums are carried in FP64 whatever the storage type.  V is a template
    // constant of the body (1, 2, 4 or 8 for every tile that fits the LDS), so
    // a thread's 2V reads are all issued before the first is used.
    const int TPP = min(NTH / P, N / 2);                     // a power of two
    const int lT = 31 - __clz(TPP);
    auto separate = [&](auto vc) {
        constexpr int V = decltype(vc)::value;
        const int W = min(TPP, 64);                          // scan width inside a wavefront
        const int p = tid >> lT, t = tid & (TPP - 1), tw = t & (W - 1);
        double ra[V], rb[V];
        double ta = 0.0, tb = 0.0;
        // slots of k = t V + e and of its partner N - k: t V and N - (t+1) V are
        // multiples of V <= 8, so with 16-byte pairs the slot moves by e (by V - e
        // from the partners' block; e = 0 has the next block's first element)
        const int ak = zsp<T, P>(p, t * V), an = zsp<T, P>(p, (N - (t + 1) * V) & (N - 1)),
                  a0n = zsp<T, P>(p, (N - t * V) & (N - 1));
        auto slot_k = [&](int e) { return sizeof(T) == 8 ? ak ^ e : zsp<T, P>(p, t * V + e); };
        auto slot_n = [&](int e) {
            if constexpr (sizeof(T) == 8) return e == 0 ? a0n : an ^ (V - e);
            return zsp<T, P>(p, (N - t * V - e) & (N - 1));
        };
        cpx<T>* zp = z + p * NS;
        if (p < P) {
            cpx<T> Zk[V], Zn[V];
#pragma unroll
            for (int e = 0; e < V; ++e) {
                Zk[e] = zp[slot_k(e)];
                Zn[e] = zp[slot_n(e)];
            }
#pragma unroll
            for (int e = 0; e < V; ++e) {
                const int k = t * V + e;
                const T Ra = T(0.5) * (Zk[e].x + Zn[e].x), Ia = T(0.5) * (Zk[e].y - Zn[e].y);
                const T Rb = T(0.5) * (Zk[e].y + Zn[e].y), Ib = -T(0.5) * (Zk[e].x - Zn[e].x);
                if (k > 0) zp[slot_n(e)] = cpx<T>{-Ia, -Ib};
                const double h = k == 0 ? 0.5 : 1.0;
                ta += h * (double)Ra;
                tb += h * (double)Rb;
                ra[e] = ta;
                rb[e] = tb;
            }
        }
        ta = group_scan(ta, W, tid & 63);
        tb = group_scan(tb, W, tid & 63);
        double ea = dpp_f64<kDppWaveShr1>(ta), eb = dpp_f64<kDppWaveShr1>(tb);   // the lane below's
        if (tw == 0) ea = eb = 0.0;
        if (TPP > 64) {
            const int nw = TPP >> 6;                         // wavefronts per pair (<= 16)
            double2* tot = reinterpret_cast<double2*>(smem_d);
            if (p < P && (t & 63) == 63) tot[p * nw + (t >> 6)] = make_double2(ta, tb);
            __syncthreads();
            if (p < P) {
                // the earlier wavefronts' totals in order; four reads issued
                // together (clamped to the pair's entries), the later ones skipped
                const int wt = t >> 6;
                double ba = 0.0, bb = 0.0;
                for (int w0 = 0; w0 < nw; w0 += 4) {
                    double2 tv[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) tv[u] = tot[p * nw + min(w0 + u, nw - 1)];
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        if (w0 + u < wt) {
                            ba += tv[u].x;
                            bb += tv[u].y;
                        }
                }
                ea += ba;
                eb += bb;
            }
        }
        if (p < P) {
#pragma unroll
            for (int e = 0; e < V; ++e) zp[slot_k(e)] = cpx<T>{(T)(ea + ra[e]), (T)(eb + rb[e])};
        }
    };
    switch ((N / 2) >> lT) {                                 // dst_tile_ok admits V <= 8 only
        case 1: separate(IntConst<1>{}); break;
        case 2: separate(IntConst<2>{}); break;
        case 4: separate(IntConst<4>{}); break;
        default: separate(IntConst<8>{}); break;
    }
    __syncthreads();
    // write: X_l to row l-1 (odd l from slot (l-1)/2, even l from slot N - l/2); row N-1 is the pad
    // (every thread reads LDS and, when accumulating, loads the old values at a
    // valid place: clamped past the tile's last element, only the stores are
    // guarded, so the reads of a batch issue together)
    for (int base = 0; base < N * P; base += NTH * kLoadBatch) {
        double vx[kLoadBatch], vy[kLoadBatch];
        cpx<T> ev[kLoadBatch];
#pragma unroll
        for (int u = 0; u < kLoadBatch; ++u) {
            const int idx = min(base + u * NTH + tid, N * P - 1);
            const int r = idx >> LP, p = idx & (P - 1);
            const int l = r + 1;                             // l = N: slot N/2, not used
            ev[u] = z[p * NS + zsp<T, P>(p, (l & 1) ? (l - 1) >> 1 : N - (l >> 1))];
        }
#pragma unroll
        for (int u = 0; u < kLoadBatch; ++u) {
            const int l = (min(base + u * NTH + tid, N * P - 1) >> LP) + 1;
            vx[u] = l < N ? alpha * (double)ev[u].x : 0.0;
            vy[u] = l < N ? alpha * (double)ev[u].y : 0.0;
        }
        if (accumulate) {
            Vout old[kLoadBatch];
#pragma unroll
            for (int u = 0; u < kLoadBatch; ++u) {
                const int idx = min(base + u * NTH + tid, N * P - 1);
                const int r = idx >> LP, p = idx & (P - 1);
                old[u] = *reinterpret_cast<const Vout*>(out + (size_t)r * ld + col0 + 2 * p);
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

// The value of lane ^ s (s = 1, 2, 4, 8, 16 or 32; every lane active) without
// a round trip through LDS: DPP quad swaps for 1 and 2, the row shifts left
// and right by 4 (each lane takes the one that stays in its half-row) for 4,
// the row rotation by 8 for 8, and gfx950's permlane swaps for 16 (odd rows
// take the first result, even rows the second) and 32 (the upper half the
// first, the lower half the second).
constexpr int kDppRowRor8 = 0x128;                           // rotate right by 8 inside each row of 16 lanes
__device__ __forceinline__ int lane_xor_i32(int v, int s, int lane) {
    switch (s) {
        case 1: return __builtin_amdgcn_update_dpp(0, v, kDppQuadSwap1, 0xf, 0xf, false);
        case 2: return __builtin_amdgcn_update_dpp(0, v, kDppQuadSwap2, 0xf, 0xf, false);
        case 4: {
            const int l = __builtin_amdgcn_update_dpp(0, v, kDppRowShl1 + 3, 0xf, 0xf, false);
            const int r = __builtin_amdgcn_update_dpp(0, v, kDppRowShr1 + 3, 0xf, 0xf, false);
            return (lane & 4) ? r : l;
        }
        case 8: return __builtin_amdgcn_update_dpp(0, v, kDppRowRor8, 0xf, 0xf, false);
        case 16: {
            const auto p = __builtin_amdgcn_permlane16_swap((unsigned)v, (unsigned)v, false, false);
            return (int)((lane & 16) ? p[0] : p[1]);
        }
        default: {
            const auto p = __builtin_amdgcn_permlane32_swap((unsigned)v, (unsigned)v, false, false);
            return (int)((lane & 32) ? p[0] : p[1]);
        }
    }
}

__device__ __forceinline__ double lane_xor(double v, int s, int lane) {
    return __hiloint2double(lane_xor_i32(__double2hiint(v), s, lane), lane_xor_i32(__double2loint(v), s, lane));
}

// Column sine transforms of short columns, N = 64 NP (NP = 1, 2 or 4; the
// dispatch uses NP = 1): one wavefront per column pair, in registers, with the same DST-I through one
// complex FFT per pair as above.  Lane L holds the points L + 64 r (r < NP).
// The FFT is decimation in frequency on the natural order: the stages at
// half-sizes N/2 .. 64 pair registers of a lane, the stages at 32 .. 1 pair
// lanes (exchanged across the wavefront), and point p ends up holding the
// transform at frequency rev(p).  Lane L then takes Z_k and Z_{N-k} for
// k = L + 64 t (t < NP/2; with NP = 1 the lanes below 32), separates the pair
// and sums the odd outputs with a wavefront scan.  No LDS but the 16-byte
// quarter-period twiddle table, no barrier after it.
constexpr int kShortThreads = 256;   // four pairs (eight columns) per workgroup

template <int NP>
__global__ __launch_bounds__(kShortThreads) void k_dst_short(const double* __restrict__ sinq, const double* in,
                                                             double* out, double alpha, int accumulate, int ld,
                                                             size_t slice, const int* __restrict__ skip) {
    constexpr int N = 64 * NP;
    constexpr int LOG2N = NP == 1 ? 6 : NP == 2 ? 7 : 8;
    constexpr int KT = NP >= 2 ? NP / 2 : 1;                 // values of k per lane
    if (skip && *skip) return;
    // tiles of eight columns (64 bytes of a row, half a cache line), in all
    // slices: consecutive workgroups go round-robin over the 8 XCDs, so each
    // XCD takes a contiguous range of the flattened (slice, tile) order and
    // neighbouring tiles share their lines in its L2
    const int Gx = gridDim.x, Gt = Gx * gridDim.y;
    int lin = (int)blockIdx.x + (int)blockIdx.y * Gx;
    if ((Gt & 7) == 0) lin = (lin & 7) * (Gt >> 3) + (lin >> 3);
    const int tile = lin % Gx;
    in += (size_t)(lin / Gx) * slice;
    out += (size_t)(lin / Gx) * slice;
    __shared__ cpx<double> tw[N / 4];
    const int tid = threadIdx.x, L = tid & 63;
    for (int k = tid; k < N / 4; k += kShortThreads) tw[k] = cpx<double>{sinq[N / 2 - 2 * k], -sinq[2 * k]};
    const int col = 8 * tile + 2 * (tid >> 6);
    // load and pre-process: y_j = sin(pi j/N)(x_j + x_{N-j}) + (x_j - x_{N-j})/2, y_0 = 0
    cpx<double> v[NP];
    {
        double2 xa[NP], xb[NP];
        double sj[NP];
#pragma unroll
        for (int r = 0; r < NP; ++r) {
            const int j = L + 64 * r;
            xa[r] = xb[r] = make_double2(0.0, 0.0);
            if (j >= 1) {
                xa[r] = *reinterpret_cast<const double2*>(in + (size_t)(j - 1) * ld + col);
                xb[r] = *reinterpret_cast<const double2*>(in + (size_t)(N - j - 1) * ld + col);
            }
            sj[r] = sinq[min(j, N - j)];
        }
#pragma unroll
        for (int r = 0; r < NP; ++r) {
            const double s = sj[r];
            v[r] = cpx<double>{s * (xa[r].x + xb[r].x) + 0.5 * (xa[r].x - xb[r].x),
                               s * (xa[r].y + xb[r].y) + 0.5 * (xa[r].y - xb[r].y)};
        }
    }
    __syncthreads();                                         // the twiddle table
    auto twid = [&](int k) {                                 // W_N^k, 0 <= k < N/2
        const cpx<double> w = tw[k & (N / 4 - 1)];
        return (k & (N / 4)) ? cpx<double>{w.y, -w.x} : w;
    };
    auto cmul = [](cpx<double> a, cpx<double> w) {
        return cpx<double>{a.x * w.x - a.y * w.y, a.x * w.y + a.y * w.x};
    };
    // stages inside a lane: half-size N/2 .. 64 (register distance half/64)
#pragma unroll
    for (int half = N / 2; half >= 64; half /= 2) {
        const int sreg = half / 64;
#pragma unroll
        for (int r = 0; r < NP; ++r) {
            if ((r / sreg) % 2 == 0) {
                const int q = (L + 64 * r) & (half - 1);
                const cpx<double> a = v[r], b = v[r + sreg];
                v[r] = cpx<double>{a.x + b.x, a.y + b.y};
                v[r + sreg] = cmul(cpx<double>{a.x - b.x, a.y - b.y}, twid(q * (N / (2 * half))));
            }
        }
    }
    // stages across lanes: half-size 32 .. 1
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) {
        const bool up = (L & s) != 0;
        const cpx<double> w = twid((L & (s - 1)) * (N / (2 * s)));
#pragma unroll
        for (int r = 0; r < NP; ++r) {
            const cpx<double> o{lane_xor(v[r].x, s, L), lane_xor(v[r].y, s, L)};
            v[r] = up ? cmul(cpx<double>{o.x - v[r].x, o.y - v[r].y}, w) : cpx<double>{v[r].x + o.x, v[r].y + o.y};
        }
    }
    // Z_k sits at point rev(k): lane rev(k) & 63, register rev(k) >> 6
    auto fetch = [&](int k) {
        const int pk = (int)(__brev((unsigned)k) >> (32 - LOG2N));
        const int src = pk & 63, reg = pk >> 6;
        cpx<double> z{0.0, 0.0};
#pragma unroll
        for (int r = 0; r < NP; ++r) {
            const double zx = __shfl(v[r].x, src, 64), zy = __shfl(v[r].y, src, 64);
            if (r == reg) z = cpx<double>{zx, zy};
        }
        return z;
    };
    double pa[KT], pb[KT], ia[KT], ib[KT];
#pragma unroll
    for (int t = 0; t < KT; ++t) {
        const int k = L + 64 * t;
        const cpx<double> Zk = fetch(k), Zn = fetch((N - k) & (N - 1));
        const double h = k == 0 ? 0.5 : 1.0;
        pa[t] = h * 0.5 * (Zk.x + Zn.x);
        pb[t] = h * 0.5 * (Zk.y + Zn.y);
        ia[t] = 0.5 * (Zk.y - Zn.y);
        ib[t] = -0.5 * (Zk.x - Zn.x);
    }
    // odd outputs: inclusive scan over k (each t across the lanes, then the
    // earlier segments' totals in order)
    double ca = 0.0, cb = 0.0;
#pragma unroll
    for (int t = 0; t < KT; ++t) {
        pa[t] = group_scan(pa[t], 64, L) + ca;
        pb[t] = group_scan(pb[t], 64, L) + cb;
        ca = readlane_f64(pa[t], 63);
        cb = readlane_f64(pb[t], 63);
    }
    // write: X_{2k+1} to row 2k, X_{2k} = -I_k to row 2k-1, the pad row N-1 zero
    auto put = [&](int row, double a, double b) {
        double2* o = reinterpret_cast<double2*>(out + (size_t)row * ld + col);
        double2 val = make_double2(alpha * a, alpha * b);
        if (accumulate) {
            const double2 old = *o;
            val.x += old.x;
            val.y += old.y;
        }
        *o = val;
    };
#pragma unroll
    for (int t = 0; t < KT; ++t) {
        const int k = L + 64 * t;
        if (k < N / 2) {
            put(2 * k, pa[t], pb[t]);
            if (k > 0) put(2 * k - 1, -ia[t], -ib[t]);
            else put(N - 1, 0.0, 0.0);
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

template <int NP>
hipError_t short_launch(const Lines& g, const double* in, double* out, double alpha, bool acc, hipStream_t s) {
    constexpr int cols = 2 * (kShortThreads / 64);
    if (hipError_t e_ = klaunch(&k_dst_short<NP>, dim3(g.ld / cols, g.slices), dim3(kShortThreads), 0, s, g.sinq,
                                in, out, alpha, acc ? 1 : 0, g.ld, g.slice, g.skip))
        return e_;
    return hipGetLastError();
}

template <class T, class Tin, class Tout>
hipError_t dst_dispatch(const Lines& g, const Tin* in, Tout* out, double alpha, bool acc, int B, hipStream_t s) {
    // FP64 columns of 64 rows: one wavefront per column pair (4.6 against 7.2
    // us for the 64^3 grid's transform along z; at 128 and 256 rows the tiled
    // kernel is the faster one: 12.0 against 15.5 us, 75 against 93 us)
    if constexpr (sizeof(T) == 8 && sizeof(Tin) == 8 && sizeof(Tout) == 8) {
        if (g.ld % 8 == 0 && g.N == 64) return short_launch<1>(g, in, out, alpha, acc, s);
    }
    if (!dst_tile_ok(g.N, B, sizeof(cpx<T>), ~(size_t)0) || g.ld % B != 0) return hipErrorInvalidValue;
    switch (B) {
        case 4: return dst_launch<T, Tin, Tout, 4>(g, in, out, alpha, acc, s);
        case 8: return dst_launch<T, Tin, Tout, 8>(g, in, out, alpha, acc, s);
        case 16: return dst_launch<T, Tin, Tout, 16>(g, in, out, alpha, acc, s);
        default:
            if constexpr (sizeof(T) == 8) {                  // wide tiles: 16-byte pairs only
                if (B == 32) return dst_launch<T, Tin, Tout, 32>(g, in, out, alpha, acc, s);
                return dst_launch<T, Tin, Tout, 64>(g, in, out, alpha, acc, s);
            }
            return hipErrorInvalidValue;
    }
}

Lines grid2(const DevPlan& p) { return Lines{p.N, p.log2N, p.sinq, p.N, 1, 0, nullptr}; }

}  // namespace

size_t dst_lds_bytes(int N, int B, size_t cpx_bytes) {
    const int pad = cpx_bytes == 16 ? (B == 4 ? pair_pad<double, 4>() : B == 8 ? pair_pad<double, 8>()
                                       : B == 16 ? pair_pad<double, 16>() : pair_pad<double, 32>())
                                     : 32 / (B / 2);
    static_assert(pair_pad<double, 32>() == pair_pad<double, 64>(), "one pad for the wide tiles");
    return sizeof(double) * (size_t)dst_table_len(N) + cpx_bytes * (size_t)(B / 2) * (N + pad);
}

bool dst_tile_ok(int N, int B, size_t cpx_bytes, size_t lds_max) {
    if (B < 4 || B > 64 || (B & (B - 1))) return false;
    if (B > 16 && cpx_bytes != 16) return false;             // wide tiles: 16-byte pairs only
    if (N < 32 || (N & (N - 1)) || N % B || N / 2 < 256 / B) return false;
    const int P = B / 2;
    if ((N / 2) / std::min(kDstThreads / P, N / 2) > 8) return false;   // the scan's values per thread
    return dst_lds_bytes(N, B, cpx_bytes) <= lds_max;
}

int dst_default_tile(int N, size_t cpx_bytes, size_t lds_max, long lines, int min_groups) {
    // the widest valid tile that still gives min_groups workgroups (wider
    // tiles read longer row segments and keep more of a workgroup's threads
    // busy in the passes; more workgroups fill the chip); else the narrowest
    // valid one
    for (int B : {64, 32, 16, 8, 4})
        if (dst_tile_ok(N, B, cpx_bytes, lds_max) && lines / B >= min_groups) return B;
    for (int B : {4, 8, 16, 32, 64})
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
