// Host-side geometry plan (see plan.h).  Readings where the paper is silent:
//  - Gamma is the periodic cubic spline through the samples in the sample index.
//  - Nodes are classified along horizontal grid lines: a node within 1e-10 h of
//    a crossing lies on Gamma and counts as inside; otherwise it is inside when
//    an odd number of crossings lie to its left.
//  - An edge whose end nodes differ must hold exactly one crossing; no edge may
//    hold a crossing strictly inside while its end nodes agree; the curve keeps
//    2h away from the box.
//  - The interpolation stencil is the 5-point cross around the nearest node plus
//    the diagonal node towards the sample (Alg. 3, six points).
#include "plan.h"

#include <algorithm>
#include <cmath>
#include <cstdio>

namespace kfbi {

namespace {

constexpr double kSnap = 1e-10;

[[noreturn]] void fail(const char* fmt, int a = 0, int b = 0, int c = 0) {
    char buf[256];
    std::snprintf(buf, sizeof buf, fmt, a, b, c);
    throw GeometryError{buf};
}

// Cubic of one spline segment in power form: A + B u + C u^2 + D u^3.
struct Cubic {
    double A, B, C, D;
    double at(double u) const { return A + u * (B + u * (C + u * D)); }
};

Cubic segment_cubic(double y0, double y1, double s0, double s1) {
    return {y0, (y1 - y0) - s0 / 3.0 - s1 / 6.0, 0.5 * s0, (s1 - s0) / 6.0};
}

// Value, first and second derivative of the spline at (segment, u).
void eval_spline(const std::vector<double>& y, const std::vector<double>& s2, int seg, double u,
                 double& v, double& d1, double& d2) {
    const int m = (int)y.size();
    const int k1 = (seg + 1) % m;
    const double y0 = y[seg], y1 = y[k1], s0 = s2[seg], s1 = s2[k1];
    const double w = 1.0 - u;
    v = w * y0 + u * y1 + (w * w * w - w) * s0 / 6.0 + (u * u * u - u) * s1 / 6.0;
    d1 = (y1 - y0) - (3.0 * w * w - 1.0) * s0 / 6.0 + (3.0 * u * u - 1.0) * s1 / 6.0;
    d2 = w * s0 + u * s1;
}

struct Crossing {
    int line;     // grid line index
    int seg;
    double u;
    double pos;   // coordinate along the line
};

// All crossings of one coordinate of the curve with the levels lo + k h.
// Every segment is cut at the zeros of its derivative into monotone pieces; a
// piece owns the levels of its half-open value range that contains its start,
// so a crossing at a sample is counted once (by the segment starting there).
std::vector<Crossing> crossings(const std::vector<double>& c, const std::vector<double>& s2,
                                const std::vector<double>& other, const std::vector<double>& os2,
                                int n, double lo, double h) {
    const int m = (int)c.size();
    std::vector<Crossing> out;
    for (int seg = 0; seg < m; ++seg) {
        const int k1 = (seg + 1) % m;
        const Cubic cb = segment_cubic(c[seg], c[k1], s2[seg], s2[k1]);
        // derivative B + 2C u + 3D u^2: stable quadratic roots
        double r[2];
        int nr = 0;
        const double qa = 3.0 * cb.D, qb = 2.0 * cb.C, qc = cb.B;
        if (qa != 0.0) {
            const double disc = qb * qb - 4.0 * qa * qc;
            if (disc >= 0.0) {
                const double sq = std::sqrt(disc);
                const double q = -0.5 * (qb + (qb >= 0 ? sq : -sq));
                if (q != 0.0) {
                    r[nr++] = q / qa;
                    r[nr++] = qc / q;
                } else {
                    r[nr++] = 0.0;
                }
            }
        } else if (qb != 0.0) {
            r[nr++] = -qc / qb;
        }
        double cut[4];
        int nc = 0;
        cut[nc++] = 0.0;
        if (nr == 2 && r[0] > r[1]) std::swap(r[0], r[1]);
        for (int k = 0; k < nr; ++k)
            if (r[k] > 0.0 && r[k] < 1.0) cut[nc++] = r[k];
        cut[nc++] = 1.0;
        for (int p = 0; p + 1 < nc; ++p) {
            const double a = cut[p], b = cut[p + 1];
            const double fa = (p == 0) ? c[seg] : cb.at(a);
            const double fb = (p + 2 == nc) ? c[k1] : cb.at(b);
            if (fa == fb) continue;
            const bool up = fb > fa;
            const double vmin = up ? fa : fb, vmax = up ? fb : fa;
            int klo = (int)std::floor((vmin - lo) / h) - 1;
            int khi = (int)std::ceil((vmax - lo) / h) + 1;
            klo = std::max(klo, 0);
            khi = std::min(khi, n);
            for (int k = klo; k <= khi; ++k) {
                const double lev = lo + k * h;
                const bool own = up ? (lev >= fa && lev < fb) : (lev <= fa && lev > fb);
                if (!own) continue;
                double u;
                if (lev == fa) {
                    u = a;
                } else {
                    double L = a, R = b;
                    for (int it = 0; it < 100; ++it) {
                        const double mid = 0.5 * (L + R);
                        if (!(mid > L && mid < R)) break;
                        const bool below = cb.at(mid) < lev;
                        if (below == up) L = mid; else R = mid;
                    }
                    u = 0.5 * (L + R);
                }
                double v, d1, d2;
                eval_spline(other, os2, seg, u, v, d1, d2);
                out.push_back({k, seg, u, v});
            }
        }
    }
    return out;
}

PointGeom geom_at(const Plan& P, int seg, double u) {
    double x, x1, x2, y, y1, y2;
    eval_spline(P.px, P.sx2, seg, u, x, x1, x2);
    eval_spline(P.py, P.sy2, seg, u, y, y1, y2);
    const double s2 = x1 * x1 + y1 * y1;
    const double s = std::sqrt(s2);
    PointGeom g;
    g.seg = seg;
    g.u = u;
    g.tx = x1 / s;
    g.ty = y1 / s;
    g.nx = g.ty;
    g.ny = -g.tx;
    g.curv = (x1 * y2 - y1 * x2) / (s2 * s);
    g.a1 = 1.0 / s;
    g.a2 = 1.0 / s2;
    g.a3 = (x1 * x2 + y1 * y2) / (s2 * s2);
    return g;
}

}  // namespace

void periodic_spline(const double* y, int m, double* s2) {
    // s[k-1] + 4 s[k] + s[k+1] = 6 (y[k+1] - 2 y[k] + y[k-1]), periodic.
    // Split off the two corner entries as a rank-one term (Sherman-Morrison)
    // and solve the remaining tridiagonal systems by elimination.
    std::vector<double> rhs(m), diag(m, 4.0), u(m, 0.0), yv(m), zv(m), cp(m);
    for (int k = 0; k < m; ++k)
        rhs[k] = 6.0 * (y[(k + 1) % m] - 2.0 * y[k] + y[(k + m - 1) % m]);
    const double gamma = -4.0;
    diag[0] -= gamma;                 // 8
    diag[m - 1] -= 1.0 / gamma;       // 4.25
    u[0] = gamma;
    u[m - 1] = 1.0;
    auto tri = [&](const std::vector<double>& d, std::vector<double>& x) {
        // forward elimination with unit off-diagonals
        cp[0] = 1.0 / diag[0];
        x[0] = d[0] / diag[0];
        for (int k = 1; k < m; ++k) {
            const double den = diag[k] - cp[k - 1];
            cp[k] = 1.0 / den;
            x[k] = (d[k] - x[k - 1]) / den;
        }
        for (int k = m - 2; k >= 0; --k) x[k] -= cp[k] * x[k + 1];
    };
    tri(rhs, yv);
    tri(u, zv);
    const double vy = yv[0] + yv[m - 1] / gamma;
    const double vz = zv[0] + zv[m - 1] / gamma;
    const double f = vy / (1.0 + vz);
    for (int k = 0; k < m; ++k) s2[k] = yv[k] - f * zv[k];
}

std::vector<double> spline_filter_taps(int K) {
    // inverse of the infinite (1, 4, 1) Toeplitz operator: g_k = rho^|k| / (2 sqrt 3),
    // rho = sqrt(3) - 2; taps of s2 = 6 g * (second difference of y).
    const double rho = std::sqrt(3.0) - 2.0;
    auto g = [&](int k) { k = std::abs(k); return k > K ? 0.0 : std::pow(rho, k) / (2.0 * std::sqrt(3.0)); };
    std::vector<double> c(2 * K + 3);
    for (int q = -K - 1; q <= K + 1; ++q) c[q + K + 1] = 6.0 * (g(q - 1) - 2.0 * g(q) + g(q + 1));
    return c;
}

Plan build_plan(const double* xy, int m, int n, double lo, double hi) {
    Plan P;
    P.n = n;
    P.M = m;
    P.lo = lo;
    P.hi = hi;
    P.h = (hi - lo) / n;
    const double h = P.h, eps = kSnap * P.h;
    P.px.resize(m);
    P.py.resize(m);
    for (int k = 0; k < m; ++k) {
        P.px[k] = xy[2 * k];
        P.py[k] = xy[2 * k + 1];
        if (!std::isfinite(P.px[k]) || !std::isfinite(P.py[k])) fail("non-finite boundary sample %d", k);
    }
    P.sx2.resize(m);
    P.sy2.resize(m);
    periodic_spline(P.px.data(), m, P.sx2.data());
    periodic_spline(P.py.data(), m, P.sy2.data());

    // crossings with lines y = y_j (varying x) and x = x_i (varying y)
    std::vector<Crossing> ch = crossings(P.py, P.sy2, P.px, P.sx2, n, lo, h);
    std::vector<Crossing> cv = crossings(P.px, P.sx2, P.py, P.sy2, n, lo, h);
    if (ch.empty()) fail("the curve crosses no grid line");

    const double mlo = lo + 2.0 * h, mhi = hi - 2.0 * h;
    for (const auto& c : ch)
        if (c.pos < mlo || c.pos > mhi) fail("curve within 2h of the box (line y_%d)", c.line);
    for (const auto& c : cv)
        if (c.pos < mlo || c.pos > mhi) fail("curve within 2h of the box (line x_%d)", c.line);
    for (int k = 0; k < m; ++k)
        if (P.px[k] < mlo || P.px[k] > mhi || P.py[k] < mlo || P.py[k] > mhi)
            fail("boundary sample %d within 2h of the box", k);

    // bucket the crossings per line, sorted by position
    auto bucket = [&](std::vector<Crossing>& cs) {
        std::sort(cs.begin(), cs.end(), [](const Crossing& a, const Crossing& b) {
            return a.line != b.line ? a.line < b.line : a.pos < b.pos;
        });
        std::vector<int> ptr(n + 2, 0);
        for (const auto& c : cs) ptr[c.line + 1]++;
        for (int k = 0; k <= n; ++k) ptr[k + 1] += ptr[k];
        return ptr;
    };
    std::vector<int> hp = bucket(ch), vp = bucket(cv);

    // classification along horizontal lines: node x_i is in Omega when an odd
    // number of the line's crossings lie strictly left of it, or when it lies
    // within eps of a crossing.  Only the nodes between the first and the last
    // crossing (and within eps of them) can be inside, so only those are visited.
    const int W = n + 1;
    P.inside.assign((size_t)W * W, 0);
    int bi0 = n + 1, bi1 = -1, bj0 = n + 1, bj1 = -1;   // bounding box of the nodes in Omega
    for (int j = 0; j <= n; ++j) {
        const int b = hp[j], e = hp[j + 1];
        if ((e - b) % 2) fail("odd number of crossings on line y_%d", j);
        if (e == b) continue;
        const int i_lo = std::max(0, (int)std::floor((ch[b].pos - eps - lo) / h) - 1);
        const int i_hi = std::min(n, (int)std::ceil((ch[e - 1].pos + eps - lo) / h) + 1);
        int k = b;   // first crossing not left of the current node
        unsigned char* row = &P.inside[(size_t)j * W];
        for (int i = i_lo; i <= i_hi; ++i) {
            const double x = lo + i * h;
            while (k < e && ch[k].pos < x) ++k;
            bool on = false;
            if (k < e && std::fabs(ch[k].pos - x) <= eps) on = true;
            if (k > b && std::fabs(ch[k - 1].pos - x) <= eps) on = true;
            const int left = k - b;
            row[i] = (on || (left & 1)) ? 1 : 0;
            if (row[i]) {
                bi0 = std::min(bi0, i);
                bi1 = std::max(bi1, i);
                bj0 = std::min(bj0, j);
                bj1 = std::max(bj1, j);
            }
        }
    }
    // class changes can only sit on edges touching the box (rows and columns
    // bj0-1 .. bj1+1 and bi0-1 .. bi1+1, clamped to the grid)
    const int ei0 = std::max(0, bi0 - 1), ei1 = std::min(n, bi1 + 1);
    const int ej0 = std::max(0, bj0 - 1), ej1 = std::min(n, bj1 + 1);
    auto in = [&](int i, int j) { return P.inside[(size_t)j * W + i] != 0; };

    // crossings that belong to edges whose end nodes differ
    for (int ax = 0; ax < 2; ++ax) {
        const std::vector<Crossing>& cs = ax == 0 ? ch : cv;
        const std::vector<int>& ptr = ax == 0 ? hp : vp;
        // the edges whose end nodes differ, as (line, edge) in line then edge
        // order; the mask is read row by row (vertical edges compare two rows)
        std::vector<std::pair<int, int>> diff;
        const unsigned char* msk = P.inside.data();
        if (ax == 0) {
            for (int j = ej0; j <= ej1; ++j)
                for (int ed = ei0; ed < ei1; ++ed)
                    if (msk[(size_t)j * W + ed] != msk[(size_t)j * W + ed + 1]) diff.push_back({j, ed});
        } else {
            for (int ed = ej0; ed < ej1; ++ed)
                for (int i = ei0; i <= ei1; ++i)
                    if (msk[(size_t)ed * W + i] != msk[(size_t)(ed + 1) * W + i]) diff.push_back({i, ed});
            std::sort(diff.begin(), diff.end());
        }
        size_t dpos = 0;
        for (int line = 0; line <= n; ++line) {
            const int b = ptr[line], e = ptr[line + 1];
            auto cls = [&](int k) { return ax == 0 ? in(k, line) : in(line, k); };
            // same-class edges must not hold a crossing strictly inside
            for (int k = b; k < e; ++k) {
                const double pos = cs[k].pos;
                int edge = (int)std::floor((pos - lo) / h);
                for (int ed = edge - 1; ed <= edge + 1; ++ed) {
                    if (ed < 0 || ed >= n) continue;
                    const double a0 = lo + ed * h, a1 = lo + (ed + 1) * h;
                    if (cls(ed) == cls(ed + 1) && pos > a0 + eps && pos < a1 - eps)
                        fail("edge %d on line %d (axis %d) crossed twice", ed, line, ax);
                }
            }
            for (; dpos < diff.size() && diff[dpos].first == line; ++dpos) {
                const int ed = diff[dpos].second;
                const double a0 = lo + ed * h, a1 = lo + (ed + 1) * h;
                int hit = -1, cnt = 0;
                for (int k = b; k < e; ++k) {
                    if (cs[k].pos >= a0 - eps && cs[k].pos <= a1 + eps) {
                        if (hit < 0) hit = k;
                        ++cnt;
                    }
                }
                if (cnt != 1) fail("edge %d on line %d holds %d crossings", ed, line, cnt);
                const Crossing& c = cs[hit];
                P.q_axis.push_back(ax);
                P.q_t.push_back(c.seg + c.u);
                if (ax == 0) {
                    P.q_x.push_back(c.pos);
                    P.q_y.push_back(lo + line * h);
                    P.q_nodes.insert(P.q_nodes.end(), {ed, line, ed + 1, line});
                } else {
                    P.q_x.push_back(lo + line * h);
                    P.q_y.push_back(c.pos);
                    P.q_nodes.insert(P.q_nodes.end(), {line, ed, line, ed + 1});
                }
                P.q_geo.push_back(geom_at(P, c.seg, c.u));
            }
        }
    }
    const int Q = (int)P.q_axis.size();

    // irregular nodes and their arms: each crossing gives an arm to both end
    // nodes of its edge; the arms are grouped by node, nodes ordered by column
    // i then row j, a node's arms in crossing order
    struct Arm {
        long node;      // i W + j: column-major order
        int q;
        double d;
    };
    std::vector<Arm> arms;
    arms.reserve(2 * (size_t)Q);
    for (int k = 0; k < Q; ++k) {
        const int ax = P.q_axis[k];
        const int* nd = &P.q_nodes[4 * k];
        const double qpos = ax == 0 ? P.q_x[k] : P.q_y[k];
        for (int side = 0; side < 2; ++side) {
            const int mi = nd[2 * side], mj = nd[2 * side + 1];
            const int oi = nd[2 * (1 - side)], oj = nd[2 * (1 - side) + 1];
            const double other = lo + (ax == 0 ? oi : oj) * h;
            arms.push_back({(long)mi * W + mj, k, other - qpos});
        }
    }
    std::stable_sort(arms.begin(), arms.end(), [](const Arm& a, const Arm& b) { return a.node < b.node; });
    P.col_ptr.assign(n + 2, 0);
    for (size_t a0 = 0; a0 < arms.size();) {
        size_t a1 = a0;
        while (a1 < arms.size() && arms[a1].node == arms[a0].node) ++a1;
        const int i = (int)(arms[a0].node / W), j = (int)(arms[a0].node % W);
        if (a1 - a0 > 4) fail("node (%d,%d) has more than four arms", i, j);
        P.irr_i.push_back(i);
        P.irr_j.push_back(j);
        P.irr_s.push_back(in(i, j) ? 1.0 : -1.0);
        for (size_t s = 0; s < 4; ++s) {
            P.arm_q.push_back(a0 + s < a1 ? arms[a0 + s].q : -1);
            P.arm_d.push_back(a0 + s < a1 ? arms[a0 + s].d : 0.0);
        }
        P.col_ptr[i + 1]++;
        a0 = a1;
    }
    for (int i = 0; i <= n; ++i) P.col_ptr[i + 1] += P.col_ptr[i];

    // interpolation stencils at the samples
    for (int k = 0; k < m; ++k) {
        const double zx = P.px[k], zy = P.py[k];
        const int i0 = (int)std::floor((zx - lo) / h + 0.5);
        const int j0 = (int)std::floor((zy - lo) / h + 0.5);
        const int sx = zx >= lo + i0 * h ? 1 : -1;
        const int sy = zy >= lo + j0 * h ? 1 : -1;
        const double X = (zx - (lo + i0 * h)) / h, Y = (zy - (lo + j0 * h)) / h;
        const double Pm = X * Y * sx * sy;
        // weights of C, E, W, N, S, D in the quadratic through the six values
        const double w[6] = {1.0 - X * X - Y * Y + Pm,
                             0.5 * X + 0.5 * X * X - 0.5 * Pm * (sx + 1),
                             -0.5 * X + 0.5 * X * X + 0.5 * Pm * (sx - 1),
                             0.5 * Y + 0.5 * Y * Y - 0.5 * Pm * (sy + 1),
                             -0.5 * Y + 0.5 * Y * Y + 0.5 * Pm * (sy - 1),
                             Pm};
        // weights of its derivatives along x and y (in units of h) at the sample:
        // the quadratic is a + b X + c Y + d X^2 + e X Y + f Y^2 with
        // b = (E - W)/2, c = (N - S)/2, d = (E + W)/2 - C, f = (N + S)/2 - C and
        // e = sx sy (D + C - E (sx+1)/2 + W (sx-1)/2 - N (sy+1)/2 + S (sy-1)/2)
        const double sg = sx * sy;
        const double wx[6] = {-2.0 * X + sg * Y,
                              0.5 + X - 0.5 * sg * Y * (sx + 1),
                              -0.5 + X + 0.5 * sg * Y * (sx - 1),
                              -0.5 * sg * Y * (sy + 1),
                              0.5 * sg * Y * (sy - 1),
                              sg * Y};
        const double wy[6] = {-2.0 * Y + sg * X,
                              -0.5 * sg * X * (sx + 1),
                              0.5 * sg * X * (sx - 1),
                              0.5 + Y - 0.5 * sg * X * (sy + 1),
                              -0.5 + Y + 0.5 * sg * X * (sy - 1),
                              sg * X};
        const PointGeom g = geom_at(P, k, 0.0);
        const int ni[6] = {i0, i0 + 1, i0 - 1, i0, i0, i0 + sx};
        const int nj[6] = {j0, j0, j0, j0 + 1, j0 - 1, j0 + sy};
        P.cp_i0.push_back(i0);
        P.cp_j0.push_back(j0);
        P.cp_sx.push_back(sx);
        P.cp_sy.push_back(sy);
        for (int s = 0; s < 6; ++s) {
            P.cp_w.push_back(w[s]);
            P.cp_wn.push_back((g.nx * wx[s] + g.ny * wy[s]) / h);
            P.cp_out.push_back(in(ni[s], nj[s]) ? 0 : 1);
        }
        P.z_geo.push_back(g);
    }
    return P;
}

}  // namespace kfbi
