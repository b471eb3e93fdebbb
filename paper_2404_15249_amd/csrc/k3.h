// Device side of the three-dimensional problem (ellipsoid, 7-point stencil).
//
// Grid layout: the interior nodes 1..N-1 of each axis in an N x N x N FP64
// array, node (i, j, k) at ((k-1) N + (j-1)) N + (i-1); index N-1 of any axis is
// a zero pad.  Jumps at the control points are stored by component:
// J[c M + m] for c = [v], [v_x], [v_y], [v_z], [v_xx], [v_yy], [v_zz], [v_xy],
// [v_xz], [v_yz].
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.h"

namespace kfbi {

struct DevPlan3 {
    int N, log2N, M, I;
    double h, h2, kappa;
    const double* sinq;         // N/2 + 1: sin(pi k / N)
    const ModeConst* modes;     // (N-1)^2: row (k, j) of the x-solve at (k-1)(N-1) + (j-1)
    const double* geo;          // 12 M: normal, t1, t2, S11, S12, S22
    const int* fit_off;         // M + 1
    const int* fit_idx;
    const double* fit_w;        // 5 per neighbour
    const int* irr_node;        // I
    const double* irr_sign;     // I
    const int* arm_off;         // I + 1
    const int* arm_q;
    const double* arm_d;
    const int* q_axis;          // M
    const int* st_node;         // 10 M (-1: a node on the box)
    const double* st_w;         // 10 M
    const double* st_t;         // 10 M
    const unsigned char* inside;   // (N+1)^3
};

// J <- Cartesian jumps at every control point for [v] = phi, [F] = fgam (null:
// zero), [d_n v] = 0.
hipError_t launch_jumps3(const DevPlan3& p, const double* phi, const double* fgam, double* J, const int* skip,
                         hipStream_t s);
// G <- f masked to Omega (f on the (N+1)^3 grid; null: zero), in the interior layout
hipError_t launch_fill3(const DevPlan3& p, const double* f, double* G, const int* skip, hipStream_t s);
// G[node] += correction at every irregular node (Alg. 2 along the three axes)
hipError_t launch_correct3(const DevPlan3& p, const double* J, double* G, const int* skip, hipStream_t s);
// G <- (L_h - kappa)^-1 G: sine transforms along z and y, tridiagonal solves
// along x, inverse transforms (Alg. 4 in three dimensions); B: transform tile
hipError_t launch_solve3(const DevPlan3& p, double* G, int B, const int* skip, hipStream_t s);
// out[m] <- v+ at control point m (Alg. 3, ten-node stencil); with gm non-null
// (a GMRES step) the result goes to gm->w and the first Gram-Schmidt pass follows
hipError_t launch_interp3(const DevPlan3& p, const double* G, const double* J, double* out, const GmresBufs* gm,
                          hipStream_t s);
// u <- the grid solution on the (N+1)^3 grid, zero outside Omega when mask
hipError_t launch_grid_out3(const DevPlan3& p, const double* G, bool mask, double* u, hipStream_t s);

}  // namespace kfbi
