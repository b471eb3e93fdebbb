// Host driver of the geometry plans, built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_plan_asan.py.  Reads cases from
// stdin, one per line:
//   2 n lo hi m x0 y0 x1 y1 ...   (curve samples, counter-clockwise)
//   3 n lo hi a b c               (ellipsoid semi-axes)
// and prints per case "ok Q I" (2D: crossings and irregular nodes; 3D: control
// points and irregular nodes) or "geometry <message>".  Every index the plan
// stores is checked against the sizes it refers to, so a sanitizer report or a
// "bad" line names a plan that points outside its own arrays.
#include <cstdio>
#include <cstdlib>
#include <iostream>
#include <string>
#include <vector>

#include "plan.h"
#include "plan3.h"

namespace {

bool in_range(int v, int lo, int hi) { return v >= lo && v < hi; }

// one number from stdin; strtod also reads "nan" and "inf"
double rd() {
    std::string t;
    std::cin >> t;
    return std::strtod(t.c_str(), nullptr);
}

std::string check2(const kfbi::Plan& p) {
    const int n1 = p.n + 1, Q = (int)p.q_axis.size(), I = (int)p.irr_i.size();
    if ((int)p.inside.size() != n1 * n1) return "mask size";
    if ((int)p.q_nodes.size() != 4 * Q || (int)p.q_geo.size() != Q) return "crossing arrays";
    for (int q = 0; q < Q; ++q)
        for (int k = 0; k < 4; ++k)
            if (!in_range(p.q_nodes[4 * q + k], 0, n1)) return "crossing node";
    if ((int)p.arm_q.size() != 4 * I || (int)p.arm_d.size() != 4 * I) return "arm arrays";
    for (int a : p.arm_q)
        if (a != -1 && !in_range(a, 0, Q)) return "arm crossing";
    for (int k = 0; k < I; ++k)
        if (!in_range(p.irr_i[k], 1, p.n) || !in_range(p.irr_j[k], 1, p.n)) return "irregular node";
    if ((int)p.col_ptr.size() != p.n + 2 || p.col_ptr.back() != I) return "column pointers";
    if ((int)p.cp_w.size() != 6 * p.M || (int)p.z_geo.size() != p.M) return "stencil arrays";
    for (int m = 0; m < p.M; ++m)
        if (!in_range(p.cp_i0[m], 1, p.n) || !in_range(p.cp_j0[m], 1, p.n)) return "stencil centre";
    return "";
}

std::string check3(const kfbi::Plan3Host& p) {
    const int N = p.N, M = p.M(), I = p.I();
    const long cells = (long)(N - 1) * (N - 1) * (N - 1);
    if ((long)p.inside.size() != (long)(N + 1) * (N + 1) * (N + 1)) return "mask size";
    if ((int)p.pos.size() != 3 * M || (int)p.geo.size() != 12 * M) return "point arrays";
    if ((int)p.fit_off.size() != M + 1) return "fit offsets";
    for (int k : p.fit_idx)
        if (!in_range(k, 0, M)) return "fit neighbour";
    for (int v : p.irr_node)
        if (v < 0 || v >= cells) return "irregular node";
    if ((int)p.arm_off.size() != I + 1) return "arm offsets";
    for (int a : p.arm_q)
        if (!in_range(a, 0, M)) return "arm crossing";
    if ((int)p.st_node.size() != 10 * M) return "stencil arrays";
    for (int v : p.st_node)
        if (v != -1 && (v < 0 || v >= cells)) return "stencil node";
    return "";
}

}  // namespace

int main() {
    int dim;
    while (std::cin >> dim) {
        int n;
        std::cin >> n;
        const double lo = rd(), hi = rd();
        try {
            if (dim == 2) {
                int m;
                std::cin >> m;
                std::vector<double> xy(2 * (size_t)m);
                for (auto& v : xy) v = rd();
                const kfbi::Plan p = kfbi::build_plan(xy.data(), m, n, lo, hi);
                const std::string bad = check2(p);
                if (!bad.empty()) {
                    std::printf("bad %s\n", bad.c_str());
                    return 1;
                }
                std::printf("ok %d %d\n", (int)p.q_axis.size(), (int)p.irr_i.size());
            } else {
                double ax[3];
                for (auto& a : ax) a = rd();
                const kfbi::Plan3Host p = kfbi::build_plan3(n, lo, hi, ax);
                const std::string bad = check3(p);
                if (!bad.empty()) {
                    std::printf("bad %s\n", bad.c_str());
                    return 1;
                }
                std::printf("ok %d %d\n", p.M(), p.I());
            }
        } catch (const kfbi::GeometryError& e) {
            std::printf("geometry %s\n", e.msg.c_str());
        }
        std::fflush(stdout);
    }
    return 0;
}
