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

template <class T, class Tin, class Tout, int B>
__global__ __launch_bounds__(256) void k_dst_cols(int N, int log2N, const double* __restrict__ sinq,
                                                  const Tin* __restrict__ in, Tout* __restrict__ out, double alpha,
                                                  int accumulate) {
    extern __shared__ double smem_d[];
    constexpr int P = B / 2;
    const int NS = N + 1;                                    // pair stride (one pad entry)
    double* sq = smem_d;                                     // N/2 + 2
    cpx<T>* z = reinterpret_cast<cpx<T>*>(smem_d + (N / 2 + 2));   // P x NS
    const int tid = threadIdx.x;
    const int col0 = blockIdx.x * B;
    const int mask2 = 2 * N - 1;
    for (int k = tid; k <= N / 2; k += 256) sq[k] = sinq[k];
    // load: node j = r + 1 of column c at z[c/2][j] (.x even columns, .y odd);
    // kLoadBatch loads per thread are issued before any is stored, so their
    // latencies overlap
    constexpr int kLoadBatch = 16;
    for (int base = 0; base < N * B; base += 256 * kLoadBatch) {
        Tin v[kLoadBatch];
#pragma unroll
        for (int u = 0; u < kLoadBatch; ++u) {
            const int idx = base + u * 256 + tid;
            const int r = idx / B, c = idx % B;
            v[u] = (idx < N * B && r + 1 < N) ? in[(size_t)r * N + col0 + c] : Tin(0);
        }
#pragma unroll
        for (int u = 0; u < kLoadBatch; ++u) {
            const int idx = base + u * 256 + tid;
            const int r = idx / B, c = idx % B;
            if (idx < N * B && r + 1 < N) {
                cpx<T>& e = z[(c >> 1) * NS + r + 1];
                if (c & 1) e.y = (T)v[u]; else e.x = (T)v[u];
            }
        }
    }
    if (tid < P) z[tid * NS] = cpx<T>{T(0), T(0)};
    __syncthreads();
    // pre-process pairs (j, N - j)
    for (int idx = tid; idx < P * (N / 2); idx += 256) {
        const int p = idx / (N / 2), j = idx % (N / 2) + 1;         // 1 .. N/2
        cpx<T>* zp = z + p * NS;
        if (j == N / 2) {
            zp[j].x *= T(2);
            zp[j].y *= T(2);
        } else {
            const cpx<T> a = zp[j], b = zp[N - j];
            const T s = (T)sq[j];
            zp[j] = cpx<T>{s * (a.x + b.x) + T(0.5) * (a.x - b.x), s * (a.y + b.y) + T(0.5) * (a.y - b.y)};
            zp[N - j] = cpx<T>{s * (b.x + a.x) + T(0.5) * (b.x - a.x), s * (b.y + a.y) + T(0.5) * (b.y - a.y)};
        }
    }
    __syncthreads();
    // in-place radix-2 FFT: bit reversal, then log2 N butterfly passes
    for (int idx = tid; idx < P * N; idx += 256) {
        const int p = idx / N, j = idx % N;
        const int rj = bitrev(j, log2N);
        if (j < rj) {
            cpx<T>* zp = z + p * NS;
            const cpx<T> t = zp[j];
            zp[j] = zp[rj];
            zp[rj] = t;
        }
    }
    __syncthreads();
    for (int s = 1; s <= log2N; ++s) {
        const int half = 1 << (s - 1);
        for (int idx = tid; idx < P * (N / 2); idx += 256) {
            const int p = idx / (N / 2), b = idx % (N / 2);
            const int pos = b & (half - 1), grp = b >> (s - 1);
            const int i1 = grp * 2 * half + pos, i2 = i1 + half;
            const int k = pos << (log2N - s);                   // twiddle e^{-2 pi i k / N}
            const T wr = (T)sinpi_n(sq, (2 * k + N / 2) & mask2, N);
            const T wi = -(T)sinpi_n(sq, (2 * k) & mask2, N);
            cpx<T>* zp = z + p * NS;
            const cpx<T> a = zp[i1], c = zp[i2];
            const T tr = wr * c.x - wi * c.y, ti = wr * c.y + wi * c.x;
            zp[i1] = cpx<T>{a.x + tr, a.y + ti};
            zp[i2] = cpx<T>{a.x - tr, a.y - ti};
        }
        __syncthreads();
    }
    // separate the two columns: slot k <- (R_a, R_b), slot N-k <- (-I_a, -I_b) = X_2k
    for (int idx = tid; idx < P * (N / 2); idx += 256) {
        const int p = idx / (N / 2), k = idx % (N / 2);
        cpx<T>* zp = z + p * NS;
        const cpx<T> Zk = zp[k], Zn = zp[(N - k) & (N - 1)];
        const T ra = T(0.5) * (Zk.x + Zn.x), ia = T(0.5) * (Zk.y - Zn.y);
        const T rb = T(0.5) * (Zk.y + Zn.y), ib = -T(0.5) * (Zk.x - Zn.x);
        zp[k] = cpx<T>{ra, rb};
        if (k > 0) zp[N - k] = cpx<T>{-ia, -ib};
    }
    __syncthreads();
    // odd outputs: X_{2k+1} = R_0/2 + R_1 + ... + R_k, a scan per column
    {
        constexpr int TPC = 256 / B;                             // threads per column
        const int c = tid / TPC, t = tid % TPC;
        const int L = (N / 2) / TPC;                             // values per thread (>= 1)
        cpx<T>* zp = z + (c >> 1) * NS;
        const bool odd = c & 1;
        // the running sums are carried in FP64 whatever the storage type
        double run = 0.0;
        for (int q = 0; q < L; ++q) {
            const int k = t * L + q;
            double v = odd ? zp[k].y : zp[k].x;
            if (k == 0) v *= 0.5;
            run += v;
        }
        // exclusive prefix of the per-thread sums within the column's threads
        double incl = run;
        for (int off = 1; off < TPC; off <<= 1) {
            const double o = __shfl_up(incl, off, TPC);
            if (t >= off) incl += o;
        }
        double acc = incl - run;
        for (int q = 0; q < L; ++q) {
            const int k = t * L + q;
            double v = odd ? zp[k].y : zp[k].x;
            if (k == 0) v *= 0.5;
            acc += v;
            if (odd) zp[k].y = (T)acc; else zp[k].x = (T)acc;
        }
    }
    __syncthreads();
    // write: X_l to row l-1 (odd l from slot (l-1)/2, even l from slot N - l/2); row N-1 is the pad
    for (int base = 0; base < N * B; base += 256 * kLoadBatch) {
        double v[kLoadBatch];
#pragma unroll
        for (int u = 0; u < kLoadBatch; ++u) {
            const int idx = base + u * 256 + tid;
            const int r = idx / B, c = idx % B;
            const int l = r + 1;
            v[u] = 0.0;
            if (idx < N * B && l < N) {
                const cpx<T>* zp = z + (c >> 1) * NS;
                const cpx<T> e = (l & 1) ? zp[(l - 1) >> 1] : zp[N - (l >> 1)];
                v[u] = alpha * (double)((c & 1) ? e.y : e.x);
            }
        }
        if (accumulate) {
            Tout old[kLoadBatch];
#pragma unroll
            for (int u = 0; u < kLoadBatch; ++u) {
                const int idx = base + u * 256 + tid;
                old[u] = idx < N * B ? out[(size_t)(idx / B) * N + col0 + idx % B] : Tout(0);
            }
#pragma unroll
            for (int u = 0; u < kLoadBatch; ++u) v[u] += (double)old[u];
        }
#pragma unroll
        for (int u = 0; u < kLoadBatch; ++u) {
            const int idx = base + u * 256 + tid;
            if (idx < N * B) out[(size_t)(idx / B) * N + col0 + idx % B] = (Tout)v[u];
        }
    }
}

template <class T, class Tin, class Tout, int B>
hipError_t dst_launch(const DevPlan& p, const Tin* in, Tout* out, double alpha, bool acc, hipStream_t s) {
    const size_t lds = dst_lds_bytes(p.N, B, sizeof(cpx<T>));
    if (hipError_t e = hipFuncSetAttribute((const void*)k_dst_cols<T, Tin, Tout, B>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds))
        return e;
    if (hipError_t e_ = klaunch(&k_dst_cols<T, Tin, Tout, B>, dim3(p.N / B), dim3(256), lds, s, p.N, p.log2N, p.sinq, in, out, alpha, acc ? 1 : 0)) return e_;
    return hipGetLastError();
}

template <class T, class Tin, class Tout>
hipError_t dst_dispatch(const DevPlan& p, const Tin* in, Tout* out, double alpha, bool acc, int B, hipStream_t s) {
    if (!dst_tile_ok(p.N, B, sizeof(cpx<T>), ~(size_t)0)) return hipErrorInvalidValue;
    switch (B) {
        case 4: return dst_launch<T, Tin, Tout, 4>(p, in, out, alpha, acc, s);
        case 8: return dst_launch<T, Tin, Tout, 8>(p, in, out, alpha, acc, s);
        default: return dst_launch<T, Tin, Tout, 16>(p, in, out, alpha, acc, s);
    }
}

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

int dst_default_tile(int N, size_t cpx_bytes, size_t lds_max) {
    for (int B : {16, 8, 4})
        if (dst_tile_ok(N, B, cpx_bytes, lds_max)) return B;
    return 0;
}

hipError_t launch_dst_cols(const DevPlan& p, const double* in, double* out, double alpha, bool acc, int B,
                           hipStream_t s) {
    return dst_dispatch<double>(p, in, out, alpha, acc, B, s);
}

hipError_t launch_dst_cols_f32(const DevPlan& p, const double* in, float* out, double alpha, int B, hipStream_t s) {
    return dst_dispatch<float>(p, in, out, alpha, false, B, s);
}

hipError_t launch_dst_cols_f32_to64(const DevPlan& p, const float* in, double* out, double alpha, bool acc, int B,
                                    hipStream_t s) {
    return dst_dispatch<float>(p, in, out, alpha, acc, B, s);
}

}  // namespace kfbi
