// Host-side plan of the three-dimensional problem (see plan3.h for the readings).
#include "plan3.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <unordered_map>

namespace kfbi {

namespace {

[[noreturn]] void fail3(const char* msg) { throw GeometryError{msg}; }

// Solves the dense n x n system A X = B (B: n x r, row-major, overwritten by X)
// by Gaussian elimination with partial pivoting.  A is overwritten.
void solve_dense(std::vector<double>& A, std::vector<double>& B, int n, int r) {
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int i = c + 1; i < n; ++i)
            if (std::fabs(A[i * n + c]) > std::fabs(A[piv * n + c])) piv = i;
        if (A[piv * n + c] == 0.0) fail3("singular local fit (degenerate control points)");
        if (piv != c) {
            for (int k = 0; k < n; ++k) std::swap(A[c * n + k], A[piv * n + k]);
            for (int k = 0; k < r; ++k) std::swap(B[c * r + k], B[piv * r + k]);
        }
        for (int i = c + 1; i < n; ++i) {
            const double f = A[i * n + c] / A[c * n + c];
            if (f == 0.0) continue;
            for (int k = c; k < n; ++k) A[i * n + k] -= f * A[c * n + k];
            for (int k = 0; k < r; ++k) B[i * r + k] -= f * B[c * r + k];
        }
    }
    for (int c = n - 1; c >= 0; --c) {
        for (int k = 0; k < r; ++k) {
            double s = B[c * r + k];
            for (int j = c + 1; j < n; ++j) s -= A[c * n + j] * B[j * r + k];
            B[c * r + k] = s / A[c * n + c];
        }
    }
}

}  // namespace

Plan3Host build_plan3(int N, double lo, double hi, const double axes_in[3]) {
    if (N < 64 || (N & (N - 1)) != 0) fail3("3D grids need a power of two >= 64 intervals per axis");
    Plan3Host P;
    P.N = N;
    P.lo = lo;
    P.hi = hi;
    P.h = (hi - lo) / N;
    for (int a = 0; a < 3; ++a) {
        if (!(axes_in[a] > 0.0)) fail3("ellipsoid semi-axes must be positive");
        P.axes[a] = axes_in[a];
    }
    const double h = P.h;
    const double a2 = P.axes[0] * P.axes[0], b2 = P.axes[1] * P.axes[1], c2 = P.axes[2] * P.axes[2];
    const int S = N + 1;
    std::vector<double> c(S);
    for (int k = 0; k < S; ++k) c[k] = lo + (double)k * h;
    auto lin = [S](int i, int j, int k) { return ((size_t)k * S + j) * S + i; };
    P.inside.assign((size_t)S * S * S, 0);
    for (int k = 0; k < S; ++k)
        for (int j = 0; j < S; ++j)
            for (int i = 0; i < S; ++i) {
                const double x = c[i], y = c[j], z = c[k];
                const double F = x * x / a2 + y * y / b2 + z * z / c2 - 1.0;
                P.inside[lin(i, j, k)] = F < 0.0 ? 1 : 0;
            }
    for (int k = 0; k < S; ++k)
        for (int j = 0; j < S; ++j)
            for (int i = 0; i < S; ++i)
                if (P.inside[lin(i, j, k)] && (i < 2 || j < 2 || k < 2 || i > N - 2 || j > N - 2 || k > N - 2))
                    fail3("the ellipsoid must keep two grid cells away from the box");

    // crossings
    std::unordered_map<long long, int> q_of_edge;   // (axis, lower node) -> crossing
    auto edge_key = [&](int ax, size_t node) { return (long long)node * 3 + ax; };
    for (int ax = 0; ax < 3; ++ax) {
        const int o0 = ax == 0 ? 1 : 0, o1 = ax == 2 ? 1 : 2;
        const double A = P.axes[ax];
        for (int t_hi = 0; t_hi < S; ++t_hi)
            for (int t_lo = 0; t_lo < S; ++t_lo)
                for (int s = 0; s < N; ++s) {
                    int ia[3], ib[3];
                    ia[ax] = s;
                    ia[o0] = t_lo;
                    ia[o1] = t_hi;
                    ib[0] = ia[0];
                    ib[1] = ia[1];
                    ib[2] = ia[2];
                    ib[ax] = s + 1;
                    const size_t na = lin(ia[0], ia[1], ia[2]), nb = lin(ib[0], ib[1], ib[2]);
                    if (P.inside[na] == P.inside[nb]) continue;
                    const double p0 = c[t_lo] / P.axes[o0];
                    const double p1 = c[t_hi] / P.axes[o1];
                    const double rest = 1.0 - p0 * p0 - p1 * p1;
                    const double root = A * std::sqrt(std::max(rest, 0.0));
                    const double sa = c[s], sb = c[s + 1];
                    double xi = sa + sb > 0.0 ? root : -root;
                    xi = std::min(std::max(xi, sa), sb);
                    double pos[3];
                    pos[ax] = xi;
                    pos[o0] = c[t_lo];
                    pos[o1] = c[t_hi];
                    q_of_edge[edge_key(ax, na)] = P.M();
                    P.pos.insert(P.pos.end(), pos, pos + 3);
                    P.axis.push_back(ax);
                }
    }
    const int M = P.M();
    if (M < kFitMin + 1) fail3("too few crossings for the surface fits");

    // local frames: outward normal, tangent basis, second fundamental form
    P.geo.resize((size_t)12 * M);
    const double hess[3] = {2.0 / a2, 2.0 / b2, 2.0 / c2};
    for (int m = 0; m < M; ++m) {
        const double* p = &P.pos[3 * m];
        const double g[3] = {2.0 * p[0] / a2, 2.0 * p[1] / b2, 2.0 * p[2] / c2};
        const double gn = std::sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
        const double n[3] = {g[0] / gn, g[1] / gn, g[2] / gn};
        int amin = 0;
        for (int a = 1; a < 3; ++a)
            if (std::fabs(n[a]) < std::fabs(n[amin])) amin = a;
        double e[3] = {0, 0, 0};
        e[amin] = 1.0;
        double t1[3] = {e[1] * n[2] - e[2] * n[1], e[2] * n[0] - e[0] * n[2], e[0] * n[1] - e[1] * n[0]};
        const double t1n = std::sqrt(t1[0] * t1[0] + t1[1] * t1[1] + t1[2] * t1[2]);
        for (double& v : t1) v /= t1n;
        const double t2[3] = {n[1] * t1[2] - n[2] * t1[1], n[2] * t1[0] - n[0] * t1[2], n[0] * t1[1] - n[1] * t1[0]};
        double s11 = 0, s12 = 0, s22 = 0;
        for (int a = 0; a < 3; ++a) {
            s11 += t1[a] * hess[a] * t1[a];
            s12 += t1[a] * hess[a] * t2[a];
            s22 += t2[a] * hess[a] * t2[a];
        }
        double* G = &P.geo[(size_t)12 * m];
        for (int a = 0; a < 3; ++a) {
            G[a] = n[a];
            G[3 + a] = t1[a];
            G[6 + a] = t2[a];
        }
        G[9] = s11 / gn;
        G[10] = s12 / gn;
        G[11] = s22 / gn;
    }

    // weighted least-squares surface fits; neighbours found through cells of
    // size 2.5 h (a point's neighbours lie in its cell and the 26 around it)
    const double rad = 0.5 * kFitRadiusNum * h;
    const int nc = (int)std::ceil((hi - lo) / rad) + 1;
    std::unordered_map<long long, std::vector<int>> cells;
    auto cell_of = [&](const double* p, int a) { return (int)std::floor((p[a] - lo) / rad); };
    auto cell_key = [&](int x, int y, int z) { return ((long long)z * nc + y) * nc + x; };
    for (int m = 0; m < M; ++m)
        cells[cell_key(cell_of(&P.pos[3 * m], 0), cell_of(&P.pos[3 * m], 1), cell_of(&P.pos[3 * m], 2))].push_back(m);
    P.fit_off.assign(1, 0);
    std::vector<int> near;
    std::vector<double> dist;
    for (int m = 0; m < M; ++m) {
        const double* pm = &P.pos[3 * m];
        auto dist_to = [&](int k) {
            const double dx = P.pos[3 * k] - pm[0], dy = P.pos[3 * k + 1] - pm[1], dz = P.pos[3 * k + 2] - pm[2];
            return std::sqrt(dx * dx + dy * dy + dz * dz);
        };
        near.clear();
        const int cx = cell_of(pm, 0), cy = cell_of(pm, 1), cz = cell_of(pm, 2);
        for (int z = cz - 1; z <= cz + 1; ++z)
            for (int y = cy - 1; y <= cy + 1; ++y)
                for (int x = cx - 1; x <= cx + 1; ++x) {
                    auto it = cells.find(cell_key(x, y, z));
                    if (it == cells.end()) continue;
                    for (int k : it->second)
                        if (k != m && dist_to(k) <= rad) near.push_back(k);
                }
        if ((int)near.size() < kFitMin) {           // the nearest kFitMin, ties by index
            std::vector<int> all;
            for (int k = 0; k < M; ++k)
                if (k != m) all.push_back(k);
            std::stable_sort(all.begin(), all.end(), [&](int a, int b) { return dist_to(a) < dist_to(b); });
            near.assign(all.begin(), all.begin() + kFitMin);
        }
        std::sort(near.begin(), near.end());
        const int K = (int)near.size();
        const double* G = &P.geo[(size_t)12 * m];
        std::vector<double> A((size_t)K * 5), wts(K);
        for (int e = 0; e < K; ++e) {
            const int k = near[e];
            const double rel[3] = {P.pos[3 * k] - pm[0], P.pos[3 * k + 1] - pm[1], P.pos[3 * k + 2] - pm[2]};
            const double u = (rel[0] * G[3] + rel[1] * G[4] + rel[2] * G[5]) / h;
            const double v = (rel[0] * G[6] + rel[1] * G[7] + rel[2] * G[8]) / h;
            const double row[5] = {u, v, 0.5 * u * u, u * v, 0.5 * v * v};
            for (int q = 0; q < 5; ++q) A[(size_t)e * 5 + q] = row[q];
            const double d = dist_to(k) / h;
            wts[e] = 1.0 / (1.0 + d * d);
        }
        std::vector<double> Gm(25, 0.0), B((size_t)5 * K);
        for (int a = 0; a < 5; ++a) {
            for (int b = 0; b < 5; ++b) {
                double s = 0.0;
                for (int e = 0; e < K; ++e) s += A[(size_t)e * 5 + a] * wts[e] * A[(size_t)e * 5 + b];
                Gm[a * 5 + b] = s;
            }
            for (int e = 0; e < K; ++e) B[(size_t)a * K + e] = A[(size_t)e * 5 + a] * wts[e];
        }
        solve_dense(Gm, B, 5, K);
        const double scale[5] = {1.0 / h, 1.0 / h, 1.0 / (h * h), 1.0 / (h * h), 1.0 / (h * h)};
        for (int e = 0; e < K; ++e) {
            P.fit_idx.push_back(near[e]);
            for (int a = 0; a < 5; ++a) P.fit_w.push_back(B[(size_t)a * K + e] * scale[a]);
        }
        P.fit_off.push_back((int)P.fit_idx.size());
    }

    // irregular nodes and their arms, in (k, j, i) order
    P.arm_off.assign(1, 0);
    for (int k = 1; k < N; ++k)
        for (int j = 1; j < N; ++j)
            for (int i = 1; i < N; ++i) {
                const unsigned char here = P.inside[lin(i, j, k)];
                const int before = (int)P.arm_q.size();
                for (int ax = 0; ax < 3; ++ax)
                    for (int step = -1; step <= 1; step += 2) {
                        int nb[3] = {i, j, k};
                        nb[ax] += step;
                        if (P.inside[lin(nb[0], nb[1], nb[2])] == here) continue;
                        const int* low = step > 0 ? nullptr : nb;
                        const int ijk[3] = {i, j, k};
                        if (!low) low = ijk;
                        const auto it = q_of_edge.find(edge_key(ax, lin(low[0], low[1], low[2])));
                        if (it == q_of_edge.end()) fail3("internal: an arm without its crossing");
                        P.arm_q.push_back(it->second);
                        P.arm_d.push_back(c[nb[ax]] - P.pos[3 * it->second + ax]);
                    }
                if ((int)P.arm_q.size() > before) {
                    P.irr_node.push_back((k - 1) * N * N + (j - 1) * N + (i - 1));
                    P.irr_sign.push_back(here ? 1.0 : -1.0);
                    P.arm_off.push_back((int)P.arm_q.size());
                }
            }

    // interpolation stencils, weights and far-side jump coefficients
    static const int offs[kStencil3][3] = {{0, 0, 0}, {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0},
                                           {0, 0, 1}, {0, 0, -1}, {1, 1, 0}, {1, 0, 1}, {0, 1, 1}};
    P.st_node.resize((size_t)kStencil3 * M);
    P.st_w.resize((size_t)kStencil3 * M);
    P.st_t.assign((size_t)kStencil3 * M, 0.0);
    for (int m = 0; m < M; ++m) {
        const double* z = &P.pos[3 * m];
        int i0[3], sg[3];
        for (int a = 0; a < 3; ++a) {
            i0[a] = (int)std::floor((z[a] - lo) / h + 0.5);
            sg[a] = z[a] >= lo + i0[a] * h ? 1 : -1;
        }
        std::vector<double> A(kStencil3 * kStencil3), e0(kStencil3, 0.0);
        double D[kStencil3][3];
        bool out[kStencil3];
        for (int s = 0; s < kStencil3; ++s) {
            int ijk[3];
            for (int a = 0; a < 3; ++a) {
                const int o = s < 7 ? offs[s][a] : offs[s][a] * sg[a];
                ijk[a] = i0[a] + o;
                if (ijk[a] < 0 || ijk[a] > N) fail3("an interpolation stencil leaves the grid");
            }
            const bool box = ijk[0] == 0 || ijk[1] == 0 || ijk[2] == 0 || ijk[0] == N || ijk[1] == N || ijk[2] == N;
            P.st_node[(size_t)kStencil3 * m + s] =
                box ? -1 : (ijk[2] - 1) * N * N + (ijk[1] - 1) * N + (ijk[0] - 1);
            out[s] = !P.inside[lin(ijk[0], ijk[1], ijk[2])];
            for (int a = 0; a < 3; ++a) D[s][a] = lo + ijk[a] * h - z[a];
            const double x = D[s][0] / h, y = D[s][1] / h, w = D[s][2] / h;
            const double row[kStencil3] = {1.0, x, y, w, x * x, y * y, w * w, x * y, x * w, y * w};
            // A^T: column s holds the basis at node s
            for (int q = 0; q < kStencil3; ++q) A[q * kStencil3 + s] = row[q];
        }
        e0[0] = 1.0;
        solve_dense(A, e0, kStencil3, 1);
        for (int s = 0; s < kStencil3; ++s) {
            const double wt = e0[s];
            P.st_w[(size_t)kStencil3 * m + s] = wt;
            if (!out[s]) continue;
            const double dx = D[s][0], dy = D[s][1], dz = D[s][2];
            const double t[kJump3] = {1.0, dx, dy, dz, 0.5 * dx * dx, 0.5 * dy * dy, 0.5 * dz * dz,
                                      dx * dy, dx * dz, dy * dz};
            for (int q = 0; q < kJump3; ++q) P.st_t[(size_t)kJump3 * m + q] += wt * t[q];
        }
    }
    return P;
}

}  // namespace kfbi
