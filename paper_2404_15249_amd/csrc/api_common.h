// Pieces shared by the C-ABI translation units: the context, error reporting
// and graph recording.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include <cmath>

#include "graph.h"
#include "kernels.h"
#include "kfbi.h"

namespace kfbi {

// The message of the last error on this host thread (kfbi_last_error).
std::string& last_error();

inline kfbi_status set_err(kfbi_status s, const std::string& msg) {
    last_error() = msg;
    return s;
}

inline kfbi_status check_ptr(const void* p, const char* name) {
    if (!p) return set_err(KFBI_ERR_ARG, std::string(name) + " is NULL");
    return KFBI_OK;
}

// Constants of the tridiagonal solve along x of one sine mode (Alg. 4): after
// the transforms along the other axes, h^2 (L_h - kappa) acts on a row as
// v_{i-1} - (2 + d) v_i + v_{i+1}, with d = h^2 kappa + 4 sin^2 of each other
// axis' mode angle (> 0).
inline ModeConst row_solve_constants(double d, int N) {
    const int C = N / 64;
    const double sq = std::sqrt(d * (4.0 + d));
    const double r = 1.0 + 0.5 * d - 0.5 * sq;             // root of r^2 - (2 + d) r + 1 in (0, 1)
    ModeConst c{};
    c.r = r;
    c.rinv = 1.0 / r;
    c.logr = std::log1p(0.5 * d - 0.5 * sq);
    c.rC = std::pow(r, C);
    const double r2N = std::exp(2.0 * N * c.logr);
    c.smc = -r / (1.0 - r2N);
    return c;
}

// Record what `enqueue(stream)` launches as the nodes of a new graph (see
// graph.h: no stream capture) and instantiate it.  Returns false (and leaves
// *out null) if recording or instantiation fails; the caller then launches
// directly.  `enqueue` must issue kernel launches only.
template <class F>
bool record_graph(hipStream_t stream, hipGraphExec_t* out, F enqueue) {
    *out = nullptr;
    GraphRec rec;
    if (hipGraphCreate(&rec.graph, 0) != hipSuccess) {
        hipGetLastError();
        return false;
    }
    graph_rec() = &rec;
    const kfbi_status e = enqueue(stream);
    graph_rec() = nullptr;
    const bool ok = e == KFBI_OK && rec.last != nullptr &&
                    hipGraphInstantiate(out, rec.graph, nullptr, nullptr, 0) == hipSuccess;
    if (!ok) {
        hipGetLastError();
        *out = nullptr;
    }
    hipGraphDestroy(rec.graph);
    return ok;
}

}  // namespace kfbi

#define HIP_TRY(expr)                                                                                   \
    do {                                                                                                \
        hipError_t e_ = (expr);                                                                         \
        if (e_ != hipSuccess)                                                                           \
            return ::kfbi::set_err(KFBI_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

namespace kfbi {

// Arguments of one Neumann solve (device pointers, as kfbi_solve_neumann).
struct NeumannIO {
    const double *f_grid, *f_gamma, *g_n;
    double *u_grid, *u_gamma, *dn_gamma, *psi;
};

// Two Neumann solves whose problems enqueue on different streams, overlapped:
// the volume potentials, then GMRES batches on both with the host reading both
// states after each round, then the final solves.  Leaves the final solves
// enqueued (no wait at the end).  KFBI_NOT_CONVERGED if either hit its cap.
kfbi_status solve_neumann_pair(kfbi_prob* pa, const NeumannIO& ia, kfbi_prob* pb, const NeumannIO& ib, int* iters_a,
                               int* iters_b);

}  // namespace kfbi

struct kfbi_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    size_t lds_max = 65536;
    int num_cu = 256;
};
