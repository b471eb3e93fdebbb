// Host-side geometry plan of the three-dimensional problem: an ellipsoid in the
// cube [lo, hi]^3 on the N^3-interval grid, 7-point stencil.
//
// Readings where the paper is silent (it gives no three-dimensional scheme for
// the Poisson problem):
//  - Omega = { x^2/a^2 + y^2/b^2 + z^2/c^2 < 1 }; a node is inside iff that
//    level function, evaluated left to right, is negative.
//  - The control points are the crossings of the grid edges with the surface
//    (M = Q), in the order: x-edges, y-edges, z-edges; on each axis by the
//    slower other index, the faster other index, then the position on the line.
//  - Surface derivatives of the density at a control point: the quadratic in
//    tangent-plane coordinates fitted by weighted least squares (weights
//    1 / (1 + (d/h)^2)) to the other control points within 2.5 h (the 12
//    nearest if fewer), its constant term fixed at the point's own value.
//  - Interpolation: the 7-point cross around the nearest node and the diagonal
//    nodes toward the point in the xy, xz and yz planes (ten nodes, Alg. 3).
#pragma once

#include <array>
#include <vector>

#include "plan.h"

namespace kfbi {

constexpr int kFitRadiusNum = 5;    // fit radius 2.5 h = 5/2 h
constexpr int kFitMin = 12;
constexpr int kStencil3 = 10;       // interpolation nodes per control point
constexpr int kJump3 = 10;          // [v], gradient, Hessian (xx, yy, zz, xy, xz, yz)

struct Plan3Host {
    int N = 0;                      // intervals per axis (a power of two)
    double lo = 0, hi = 0, h = 0;
    std::array<double, 3> axes{};
    std::vector<unsigned char> inside;   // (N+1)^3, [k][j][i]
    // control points (= crossings)
    std::vector<double> pos;        // 3 M
    std::vector<int> axis;          // M: axis of the crossed edge
    std::vector<double> geo;        // 12 M: normal(3), t1(3), t2(3), S11, S12, S22
    // surface fit: neighbours of point m at fit_off[m] .. fit_off[m+1]
    std::vector<int> fit_off, fit_idx;
    std::vector<double> fit_w;      // 5 per neighbour: d/du, d/dv, d2/du2, d2/dudv, d2/dv2
    // irregular nodes
    std::vector<int> irr_node;      // linear index (k-1) N^2 + (j-1) N + (i-1)
    std::vector<double> irr_sign;   // +1 in Omega, -1 outside
    std::vector<int> arm_off, arm_q;
    std::vector<double> arm_d;      // coordinate of the neighbour minus that of the crossing
    // interpolation: per point ten nodes (linear index as above, -1 on the box),
    // their weights, and the jump coefficients of the far-side nodes
    std::vector<int> st_node;       // 10 M
    std::vector<double> st_w;       // 10 M
    std::vector<double> st_t;       // 10 M (dotted with the 10 jumps at the point)

    int M() const { return (int)axis.size(); }
    int I() const { return (int)irr_node.size(); }
};

// Throws GeometryError when the ellipsoid is not strictly inside the box or
// the grid is not supported.
Plan3Host build_plan3(int N, double lo, double hi, const double axes[3]);

}  // namespace kfbi
