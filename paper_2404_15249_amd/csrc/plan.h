// Host-side geometry plan of one KFBI problem (FP64).
//
// The plan is everything that depends only on the curve and the grid: the
// periodic cubic spline of Gamma, the inside/outside classification of the
// nodes, the grid-line crossings with their local geometry, the irregular
// nodes with their arms (Alg. 2), the six-point interpolation stencils and
// their weights (Alg. 3), and the per-mode constants of the fast solver
// (Alg. 4).  It is built once per problem (Sec. 4.2, Procedure 1) and uploaded.
#pragma once

#include <string>
#include <vector>

namespace kfbi {

// Local geometry of the spline curve at one parameter value, in the form the
// jump formulas consume.
struct PointGeom {
    int seg;        // spline segment [seg, seg+1)
    double u;       // offset inside the segment, 0 <= u < 1
    double tx, ty;  // unit tangent
    double nx, ny;  // unit outward normal (tangent turned clockwise)
    double curv;    // signed curvature, > 0 on convex counter-clockwise arcs
    double a1;      // 1 / |X'|
    double a2;      // 1 / |X'|^2
    double a3;      // (X' . X'') / |X'|^4
};

struct Plan {
    int n = 0, M = 0;
    double lo = 0, hi = 0, h = 0;

    std::vector<double> px, py;     // samples
    std::vector<double> sx2, sy2;   // spline second derivatives at the samples

    std::vector<unsigned char> inside;   // (n+1)^2, row j = line y_j

    // crossings
    std::vector<int> q_axis;            // 0: on a line y = y_j (edge along x), 1: on x = x_i
    std::vector<int> q_nodes;           // 4 per crossing: i0 j0 i1 j1 (lower end first)
    std::vector<double> q_t, q_x, q_y;  // parameter and position
    std::vector<PointGeom> q_geo;

    // irregular nodes, ordered by (i, j): column-major grouping by x index
    std::vector<int> irr_i, irr_j;
    std::vector<double> irr_s;           // +1 inside Omega, -1 outside
    std::vector<int> arm_q;              // 4 per node, -1 = unused
    std::vector<double> arm_d;           // 4 per node: xi(other node) - xi(crossing)
    std::vector<int> col_ptr;            // n+2: irregular nodes of column i are [col_ptr[i], col_ptr[i+1])

    // interpolation stencils at the samples
    std::vector<PointGeom> z_geo;
    std::vector<int> cp_i0, cp_j0, cp_sx, cp_sy;
    std::vector<double> cp_w;            // 6 per sample: weights of nodes C, E, W, N, S, D
    std::vector<double> cp_wn;           // 6 per sample: the same quadratic's outward normal derivative
    std::vector<unsigned char> cp_out;   // 6 per sample: 1 if that stencil node is outside Omega
};

// Throws kfbi::GeometryError with a message on unsupported geometry.
struct GeometryError {
    std::string msg;
};

Plan build_plan(const double* xy, int m, int n, double lo, double hi);

// Periodic cubic spline second derivatives through y[0..m) at t = 0..m-1.
void periodic_spline(const double* y, int m, double* s2);

// Filter taps c[-K-1 .. K+1] (stored from index 0) with s2 = sum_k c_k y[m+k].
std::vector<double> spline_filter_taps(int K);

}  // namespace kfbi
