// The other outer iterations the paper compares with GMRES (Table 2): the
// Richardson iteration of Sec. 2.1 and BiCGSTAB, on the same K_D apply.
//
// Each step between two applies is one single-workgroup kernel: the vectors
// hold at most kMaxSamples values, so 1024 threads cover them in at most 12
// strided passes, and every dot product is a fixed-order block sum (the same
// result on every run).  The scalars and the stop decision live in device
// memory (IterState), so a batch of iterations is one replayed graph and the
// host only polls between batches; once the state says done, every later
// launch of the batch returns at once.
#include <hip/hip_runtime.h>

#include "graph.h"
#include "kernels.h"

namespace kfbi {
namespace {

constexpr int kIterThreads = 1024;

// Fixed-order sum over the workgroup of up to three values per thread.
template <int K>
__device__ inline void block_sums(double (&v)[K], double* red) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
    }
    __syncthreads();
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < K; ++k) red[k * 16 + wave] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double s = 0.0;
        for (int w = 0; w < kIterThreads / 64; ++w) s += red[k * 16 + w];
        v[k] = s;
    }
    __syncthreads();
}

// Richardson, after w = K x: r = b - w and its norm; the first call sets r0.
// Converged when rel < tol after at least one update, capped at max_iter
// updates; otherwise x += gamma r for the next apply.
__global__ __launch_bounds__(kIterThreads) void k_rich_step(IterBufs B) {
    __shared__ double red[48];
    IterState* st = B.st;
    if (st->done) return;
    const int M = B.M;
    double nr[1] = {0.0};
    for (int i = threadIdx.x; i < M; i += kIterThreads) {
        const double r = B.b[i] - B.w[i];
        B.r[i] = r;
        nr[0] = fma(r, r, nr[0]);
    }
    block_sums(nr, red);
    const double norm = sqrt(nr[0]);
    const int it = st->it;
    double r0 = st->r0;
    if (it == 0 && !st->started) r0 = norm;
    const double rel = r0 > 0.0 ? norm / r0 : 0.0;
    int done = 0;
    if (!isfinite(norm)) done = kIterNonfinite;
    else if (r0 == 0.0 || (it > 0 && rel < st->tol)) done = 1;
    else if (it >= st->max_iter) done = -1;
    if (!done) {
        const double g = st->gamma;
        for (int i = threadIdx.x; i < M; i += kIterThreads) B.x[i] = fma(g, B.r[i], B.x[i]);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        st->started = 1;
        st->r0 = r0;
        st->relres = rel;
        if (!done) st->it = it + 1;
        st->done = done;
    }
}

// BiCGSTAB, after w = K x0: r = b - w, r^ = r, rho = r^.r, p = r; the next
// apply's input q = p.
__global__ __launch_bounds__(kIterThreads) void k_bicg_init(IterBufs B) {
    __shared__ double red[48];
    IterState* st = B.st;
    if (st->done) return;
    const int M = B.M;
    double nr[1] = {0.0};
    for (int i = threadIdx.x; i < M; i += kIterThreads) {
        const double r = B.b[i] - B.w[i];
        B.r[i] = r;
        B.rhat[i] = r;
        B.p[i] = r;
        B.q[i] = r;
        nr[0] = fma(r, r, nr[0]);
    }
    block_sums(nr, red);
    if (threadIdx.x == 0) {
        st->started = 1;
        st->r0 = sqrt(nr[0]);
        st->rho = nr[0];
        st->relres = nr[0] > 0.0 ? 1.0 : 0.0;
        if (!isfinite(nr[0])) st->done = kIterNonfinite;
        else if (nr[0] == 0.0) st->done = 1;
    }
}

// After v = K p: alpha = rho / (r^.v), s = r - alpha v.  Converged half way
// when |s| / r0 < tol (then x += alpha p); otherwise q = s for the next apply.
__global__ __launch_bounds__(kIterThreads) void k_bicg_half(IterBufs B) {
    __shared__ double red[48];
    IterState* st = B.st;
    if (st->done) return;
    const int M = B.M;
    double d[1] = {0.0};
    for (int i = threadIdx.x; i < M; i += kIterThreads) {
        const double v = B.w[i];
        B.v[i] = v;
        d[0] = fma(B.rhat[i], v, d[0]);
    }
    block_sums(d, red);
    if (!isfinite(d[0]) || d[0] == 0.0) {               // NaN/Inf, or breakdown: r^ orthogonal to v
        __syncthreads();
        if (threadIdx.x == 0) st->done = isfinite(d[0]) ? -1 : kIterNonfinite;
        return;
    }
    const double alpha = st->rho / d[0];
    double ns[1] = {0.0};
    for (int i = threadIdx.x; i < M; i += kIterThreads) {
        const double s = fma(-alpha, B.v[i], B.r[i]);
        B.s[i] = s;
        B.q[i] = s;
        ns[0] = fma(s, s, ns[0]);
    }
    block_sums(ns, red);
    const double rel = sqrt(ns[0]) / st->r0;
    const bool conv = rel < st->tol;
    if (conv)
        for (int i = threadIdx.x; i < M; i += kIterThreads) B.x[i] = fma(alpha, B.p[i], B.x[i]);
    __syncthreads();
    if (threadIdx.x == 0) {
        st->it = st->it + 1;
        st->alpha = alpha;
        if (conv) {
            st->relres = rel;
            st->half = 1;
            st->done = 1;
        }
    }
}

// After t = K s: omega = (t.s)/(t.t), x += alpha p + omega s, r = s - omega t.
// Converged when |r| / r0 < tol, capped at max_iter iterations; otherwise
// rho' = r^.r, p = r + (rho'/rho)(alpha/omega)(p - omega v), q = p.
__global__ __launch_bounds__(kIterThreads) void k_bicg_full(IterBufs B) {
    __shared__ double red[48];
    IterState* st = B.st;
    if (st->done) return;
    const int M = B.M;
    double d[2] = {0.0, 0.0};
    for (int i = threadIdx.x; i < M; i += kIterThreads) {
        const double t = B.w[i];
        d[0] = fma(t, B.s[i], d[0]);
        d[1] = fma(t, t, d[1]);
    }
    block_sums(d, red);
    const bool fin = isfinite(d[0]) && isfinite(d[1]);
    if (!fin || d[1] == 0.0 || d[0] == 0.0) {           // NaN/Inf, or breakdown: t = 0 or t orthogonal to s
        __syncthreads();
        if (threadIdx.x == 0) st->done = fin ? -1 : kIterNonfinite;
        return;
    }
    const double omega = d[0] / d[1], alpha = st->alpha;
    double e[2] = {0.0, 0.0};
    for (int i = threadIdx.x; i < M; i += kIterThreads) {
        const double s = B.s[i];
        B.x[i] = B.x[i] + alpha * B.p[i] + omega * s;
        const double r = fma(-omega, B.w[i], s);
        B.r[i] = r;
        e[0] = fma(r, r, e[0]);
        e[1] = fma(B.rhat[i], r, e[1]);
    }
    block_sums(e, red);
    const double rel = sqrt(e[0]) / st->r0;
    int done = 0;
    if (!isfinite(rel)) done = kIterNonfinite;
    else if (rel < st->tol) done = 1;
    else if (st->it >= st->max_iter) done = -1;
    if (!done) {
        const double beta = (e[1] / st->rho) * (alpha / omega);
        for (int i = threadIdx.x; i < M; i += kIterThreads) {
            const double pn = B.r[i] + beta * (B.p[i] - omega * B.v[i]);
            B.p[i] = pn;
            B.q[i] = pn;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        st->relres = rel;
        st->done = done;
        if (!done) st->rho = e[1];
    }
}

// The true relative residual |b - w| / r0 of the final iterate (w = K x).
__global__ __launch_bounds__(kIterThreads) void k_iter_true_res(IterBufs B) {
    __shared__ double red[48];
    double nr[1] = {0.0};
    for (int i = threadIdx.x; i < B.M; i += kIterThreads) {
        const double r = B.b[i] - B.w[i];
        nr[0] = fma(r, r, nr[0]);
    }
    block_sums(nr, red);
    if (threadIdx.x == 0) {
        const double r0 = B.st->r0;
        B.st->relres = r0 > 0.0 ? sqrt(nr[0]) / r0 : 0.0;
    }
}

}  // namespace

hipError_t launch_iter_step(int which, const IterBufs& B, hipStream_t s) {
    void (*k)(IterBufs) = which == kIterRich ? k_rich_step
                        : which == kIterBicgInit ? k_bicg_init
                        : which == kIterBicgHalf ? k_bicg_half
                        : which == kIterBicgFull ? k_bicg_full
                                                 : k_iter_true_res;
    if (hipError_t e = klaunch(k, dim3(1), dim3(kIterThreads), 0, s, B)) return e;
    return hipGetLastError();
}

}  // namespace kfbi
