// Host-side setup of libpat: P1 assembly, boundary detection, sensor location,
// node numbering and the time-step stability check.  Runs once per problem in
// float64; nothing here is on the timed path.
//
// Paper: "3D Uncertainty Quantification for Photoacoustic Tomography"
// (arXiv 2607.21373).
//   K, M, B     Sec. 3, matrices defined under eq. (semi-discrete)
//   M_L         Sec. 3, lumped mass diag(M 1)
//   Pi          Sec. 3, eq. (lagrange); sensors not at nodes use the P1
//               interpolant of the containing tetrahedron (Sec. 5.1 remark on
//               Pi^T for off-node sensors)
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <limits>
#include <thread>

#include "pat_internal.h"

namespace pat {
namespace {

// Run f(i) for i in [0, n) on up to 16 host threads (each index exactly once).
template <class F>
void parallel_for(int64_t n, F &&f) {
    unsigned nt = std::thread::hardware_concurrency();
    nt = std::max(1u, std::min(nt, 16u));
    if (n < 8192) nt = 1;
    if (nt == 1) {
        for (int64_t i = 0; i < n; ++i) f(i);
        return;
    }
    std::vector<std::thread> th;
    const int64_t chunk = (n + nt - 1) / nt;
    for (unsigned t = 0; t < nt; ++t) {
        const int64_t a = int64_t(t) * chunk, b = std::min<int64_t>(n, a + chunk);
        if (a >= b) break;
        th.emplace_back([a, b, &f] {
            for (int64_t i = a; i < b; ++i) f(i);
        });
    }
    for (auto &x : th) x.join();
}

// Shape data of one P1 tetrahedron: volume and the gradients of its four nodal
// basis functions, from the inverse of J = [x1-x0 | x2-x0 | x3-x0]: the
// barycentric coordinates are lambda_{1..3} = J^{-1} (x - x0), lambda_0 = 1 - sum.
struct Shape {
    double vol;
    double g[4][3];
    double inv[3][3];
    double x0[3];
};

bool tet_shape(const double *X, const int32_t *t, Shape &s) {
    const double *a = X + 3 * int64_t(t[0]);
    double J[3][3];
    for (int k = 0; k < 3; ++k) {
        const double *b = X + 3 * int64_t(t[k + 1]);
        for (int d = 0; d < 3; ++d) J[d][k] = b[d] - a[d];
    }
    const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                       J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                       J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    if (!(std::fabs(det) > 0.0) || !std::isfinite(det)) return false;
    const double r = 1.0 / det;
    s.inv[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) * r;
    s.inv[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * r;
    s.inv[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * r;
    s.inv[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) * r;
    s.inv[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * r;
    s.inv[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * r;
    s.inv[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) * r;
    s.inv[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * r;
    s.inv[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * r;
    for (int d = 0; d < 3; ++d) {
        s.g[1][d] = s.inv[0][d];
        s.g[2][d] = s.inv[1][d];
        s.g[3][d] = s.inv[2][d];
        s.g[0][d] = -(s.inv[0][d] + s.inv[1][d] + s.inv[2][d]);
        s.x0[d] = a[d];
    }
    s.vol = std::fabs(det) / 6.0;
    return true;
}

// Barycentric coordinates of x in the tetrahedron; returns the smallest one.
double barycentric(const Shape &s, const double *x, double lam[4]) {
    const double dx[3] = {x[0] - s.x0[0], x[1] - s.x0[1], x[2] - s.x0[2]};
    double sum = 0.0;
    for (int k = 0; k < 3; ++k) {
        lam[k + 1] = s.inv[k][0] * dx[0] + s.inv[k][1] * dx[1] + s.inv[k][2] * dx[2];
        sum += lam[k + 1];
    }
    lam[0] = 1.0 - sum;
    return std::min(std::min(lam[0], lam[1]), std::min(lam[2], lam[3]));
}

// Locality order of the nodes for the time-step kernels: recursive coordinate
// bisection (k-d order).  Each set is split at the median of its longest extent
// until it holds at most 64 nodes, and the leaves are numbered depth first.  The
// first three levels give 8 equal parts, one per XCD of the GPU; every later
// level keeps spatially close nodes close in the numbering, so a tile of
// consecutive rows touches few distinct neighbour rows and an XCD's L2 holds the
// neighbourhood of the rows it is processing.  Stable sorts keep it deterministic.
void locality_order(const double *X, int32_t N, const std::vector<char> &first, std::vector<int32_t> &perm) {
    perm.resize(size_t(N));
    for (int32_t i = 0; i < N; ++i) perm[size_t(i)] = i;
    std::vector<std::pair<size_t, size_t>> stack = {{0, size_t(N)}};
    while (!stack.empty()) {
        const auto [a, b] = stack.back();
        stack.pop_back();
        if (b - a <= 64) continue;
        double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
        for (size_t q = a; q < b; ++q)
            for (int k = 0; k < 3; ++k) {
                lo[k] = std::min(lo[k], X[3 * size_t(perm[q]) + k]);
                hi[k] = std::max(hi[k], X[3 * size_t(perm[q]) + k]);
            }
        int ax = 0;
        for (int k = 1; k < 3; ++k)
            if (hi[k] - lo[k] > hi[ax] - lo[ax]) ax = k;
        std::stable_sort(perm.begin() + a, perm.begin() + b,
                         [&](int32_t u, int32_t v) { return X[3 * size_t(u) + ax] < X[3 * size_t(v) + ax]; });
        const size_t m = a + (b - a) / 2;
        stack.push_back({m, b});
        stack.push_back({a, m});
    }
    // Within each of the eight top-level parts (one per XCD), the nodes flagged in
    // `first` (rows with a sensor weight) go to the front, each group keeping its
    // k-d order.  Those rows are few, but in plain k-d order they sit in about a
    // fifth of the tiles, and each such tile waits on the longer injection chain of
    // the transposed step; at the front of their part they fill few tiles, which are
    // also the first of that part to be dispatched.
    std::vector<std::pair<size_t, size_t>> parts = {{0, size_t(N)}};
    for (int level = 0; level < 3; ++level) {
        std::vector<std::pair<size_t, size_t>> next;
        for (const auto &[a, b] : parts) {
            if (b - a <= 64) {
                next.push_back({a, b});
                continue;
            }
            const size_t m = a + (b - a) / 2;
            next.push_back({a, m});
            next.push_back({m, b});
        }
        parts.swap(next);
    }
    for (const auto &[a, b] : parts)
        std::stable_partition(perm.begin() + a, perm.begin() + b, [&](int32_t u) { return first[size_t(u)] != 0; });
}

int local_index(const int32_t *t, int32_t node) {
    for (int a = 0; a < 4; ++a)
        if (t[a] == node) return a;
    return -1;
}

}  // namespace

pat_status build_host_problem(const pat_problem_desc &d, HostProblem &hp, std::string &err) {
    const int32_t N = d.n_nodes;
    const int64_t E = d.n_tets;
    if (N < 4 || E < 1 || !d.coords || !d.tets) {
        err = "need n_nodes >= 4, n_tets >= 1 and non-NULL coords/tets";
        return PAT_ERR_INVALID_ARG;
    }
    if (!(d.dt > 0.0) || !std::isfinite(d.dt) || d.n_steps < 1) {
        err = "dt must be positive and finite and n_steps >= 1";
        return PAT_ERR_INVALID_ARG;
    }
    if (d.n_obs < 1 || (d.sensor_nodes == nullptr) == (d.sensor_pos == nullptr)) {
        err = "need n_obs >= 1 and exactly one of sensor_nodes / sensor_pos";
        return PAT_ERR_INVALID_ARG;
    }
    for (int64_t i = 0; i < 3 * int64_t(N); ++i)
        if (!std::isfinite(d.coords[i])) {
            err = "non-finite node coordinate";
            return PAT_ERR_NONFINITE;
        }
    for (int64_t i = 0; i < 4 * E; ++i)
        if (d.tets[i] < 0 || d.tets[i] >= N) {
            err = "tetrahedron node id out of range";
            return PAT_ERR_INVALID_ARG;
        }
    if (d.c_tet)
        for (int64_t e = 0; e < E; ++e)
            if (!(d.c_tet[e] > 0.0) || !std::isfinite(d.c_tet[e])) {
                err = "wave speed must be positive and finite";
                return PAT_ERR_INVALID_ARG;
            }

    hp.n = N;
    hp.n_obs = d.n_obs;
    hp.n_steps = d.n_steps;
    hp.n_tets = E;
    hp.dt = d.dt;
    // Sensors (user numbering; mapped to the internal one further down).
    const int32_t S = d.n_obs;
    hp.snode.assign(size_t(4) * S, 0);
    hp.sw.assign(size_t(4) * S, 0.0);
    if (d.sensor_nodes) {
        for (int32_t s = 0; s < S; ++s) {
            const int32_t v = d.sensor_nodes[s];
            if (v < 0 || v >= N) {
                err = "sensor node id out of range";
                return PAT_ERR_INVALID_ARG;
            }
            for (int k = 0; k < 4; ++k) hp.snode[4 * s + k] = v;
            hp.sw[4 * s] = 1.0;
        }
    } else {
        // bucket grid over the mesh bounding box; each tetrahedron is listed in
        // every cell its bounding box touches
        double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
        for (int32_t i = 0; i < N; ++i)
            for (int k = 0; k < 3; ++k) {
                lo[k] = std::min(lo[k], d.coords[3 * i + k]);
                hi[k] = std::max(hi[k], d.coords[3 * i + k]);
            }
        const int G = std::max(1, std::min(256, int(std::cbrt(double(E) / 4.0))));
        auto cell = [&](double x, int k) {
            const double w = (hi[k] - lo[k]) > 0 ? (hi[k] - lo[k]) : 1.0;
            int c = int((x - lo[k]) / w * G);
            return std::min(G - 1, std::max(0, c));
        };
        std::vector<int64_t> cptr(size_t(G) * G * G + 1, 0);
        auto for_cells = [&](int64_t e, auto &&fn) {
            const int32_t *t = d.tets + 4 * e;
            int c0[3], c1[3];
            for (int k = 0; k < 3; ++k) {
                double a = 1e300, b = -1e300;
                for (int v = 0; v < 4; ++v) {
                    a = std::min(a, d.coords[3 * int64_t(t[v]) + k]);
                    b = std::max(b, d.coords[3 * int64_t(t[v]) + k]);
                }
                c0[k] = cell(a, k);
                c1[k] = cell(b, k);
            }
            for (int z = c0[2]; z <= c1[2]; ++z)
                for (int y = c0[1]; y <= c1[1]; ++y)
                    for (int x = c0[0]; x <= c1[0]; ++x) fn((int64_t(z) * G + y) * G + x);
        };
        for (int64_t e = 0; e < E; ++e) for_cells(e, [&](int64_t c) { ++cptr[size_t(c) + 1]; });
        for (size_t c = 0; c + 1 < cptr.size(); ++c) cptr[c + 1] += cptr[c];
        std::vector<int64_t> clist(size_t(cptr.back()));
        {
            std::vector<int64_t> fill(cptr.begin(), cptr.end() - 1);
            for (int64_t e = 0; e < E; ++e) for_cells(e, [&](int64_t c) { clist[size_t(fill[size_t(c)]++)] = e; });
        }
        int bad = -1;
        for (int32_t s = 0; s < S; ++s) {
            const double *x = d.sensor_pos + 3 * int64_t(s);
            if (!std::isfinite(x[0]) || !std::isfinite(x[1]) || !std::isfinite(x[2])) {
                bad = s;
                break;
            }
            const int64_t c = (int64_t(cell(x[2], 2)) * G + cell(x[1], 1)) * G + cell(x[0], 0);
            double best = -std::numeric_limits<double>::infinity();
            int64_t best_e = -1;
            double best_lam[4] = {0, 0, 0, 0};
            // candidates in ascending tetrahedron index; the tetrahedron whose
            // smallest barycentric coordinate is largest wins (first on ties)
            for (int64_t q = cptr[size_t(c)]; q < cptr[size_t(c) + 1]; ++q) {
                const int64_t e = clist[size_t(q)];
                Shape sh;
                tet_shape(d.coords, d.tets + 4 * e, sh);
                double lam[4];
                const double m = barycentric(sh, x, lam);
                if (m > best) {
                    best = m;
                    best_e = e;
                    std::memcpy(best_lam, lam, sizeof(lam));
                }
            }
            if (best_e < 0 || best < -1e-10) {
                bad = s;
                break;
            }
            for (int k = 0; k < 4; ++k) {
                hp.snode[4 * s + k] = d.tets[4 * best_e + k];
                hp.sw[4 * s + k] = best_lam[k];
            }
        }
        if (bad >= 0) {
            err = "sensor " + std::to_string(bad) + " is not inside the mesh";
            return PAT_ERR_INVALID_ARG;
        }
    }
    // nodes that carry a sensor weight: their rows take the injection of the transposed step
    std::vector<char> sensor_row(size_t(N), 0);
    for (size_t q = 0; q < hp.sw.size(); ++q)
        if (hp.sw[q] != 0.0) sensor_row[size_t(hp.snode[q])] = 1;

    // Internal numbering (see locality_order): perm[internal] = user node.
    locality_order(d.coords, N, sensor_row, hp.perm);
    hp.iperm.resize(N);
    for (int32_t i = 0; i < N; ++i) hp.iperm[hp.perm[i]] = i;

    // node -> incident tetrahedra (ascending tetrahedron index)
    std::vector<int64_t> inc_ptr(size_t(N) + 1, 0);
    for (int64_t i = 0; i < 4 * E; ++i) ++inc_ptr[size_t(d.tets[i]) + 1];
    for (int32_t i = 0; i < N; ++i) inc_ptr[i + 1] += inc_ptr[i];
    std::vector<int64_t> inc(static_cast<size_t>(inc_ptr[N]));
    {
        std::vector<int64_t> fill(inc_ptr.begin(), inc_ptr.end() - 1);
        for (int64_t e = 0; e < E; ++e)
            for (int a = 0; a < 4; ++a) inc[size_t(fill[d.tets[4 * e + a]]++)] = e;
    }
    for (int32_t i = 0; i < N; ++i)
        if (inc_ptr[i + 1] == inc_ptr[i]) {
            err = "node " + std::to_string(i) + " belongs to no tetrahedron";
            return PAT_ERR_INVALID_ARG;
        }

    // geometry check (no degenerate tetrahedra)
    {
        int bad = 0;
        for (int64_t e = 0; e < E && !bad; ++e) {
            Shape s;
            if (!tet_shape(d.coords, d.tets + 4 * e, s)) bad = 1;
        }
        if (bad) {
            err = "degenerate tetrahedron (zero volume)";
            return PAT_ERR_INVALID_ARG;
        }
    }

    // row pattern: all nodes that share a tetrahedron with node i
    std::vector<int32_t> rowlen(N);
    std::vector<std::vector<int32_t>> cols(N);
    parallel_for(N, [&](int64_t i) {
        const int32_t u = hp.perm[size_t(i)];
        std::vector<int32_t> &c = cols[size_t(i)];
        c.reserve(size_t(4 * (inc_ptr[u + 1] - inc_ptr[u])));
        for (int64_t q = inc_ptr[u]; q < inc_ptr[u + 1]; ++q)
            for (int a = 0; a < 4; ++a) c.push_back(hp.iperm[size_t(d.tets[4 * inc[size_t(q)] + a])]);
        std::sort(c.begin(), c.end());
        c.erase(std::unique(c.begin(), c.end()), c.end());
        rowlen[size_t(i)] = int32_t(c.size());
    });
    hp.rowptr.assign(size_t(N) + 1, 0);
    for (int32_t i = 0; i < N; ++i) {
        hp.rowptr[i + 1] = hp.rowptr[i] + rowlen[i];
        hp.max_row = std::max(hp.max_row, rowlen[i]);
    }
    const int64_t nnz = hp.rowptr[N];
    hp.col.resize(size_t(nnz));
    hp.kval.assign(size_t(nnz), 0.0);
    hp.k1val.assign(size_t(nnz), 0.0);
    hp.mass.assign(size_t(N), 0.0);

    // Stiffness rows: K_ij = sum over tetrahedra e containing i and j of
    // c_e^2 vol_e grad(phi_i).grad(phi_j); K1 the same with c = 1; M_L = sum vol_e / 4.
    parallel_for(N, [&](int64_t i) {
        const int32_t r0 = hp.rowptr[i];
        const int32_t u = hp.perm[size_t(i)];
        const std::vector<int32_t> &c = cols[size_t(i)];
        std::copy(c.begin(), c.end(), hp.col.begin() + r0);
        double m = 0.0;
        for (int64_t q = inc_ptr[u]; q < inc_ptr[u + 1]; ++q) {
            const int64_t e = inc[size_t(q)];
            const int32_t *t = d.tets + 4 * e;
            Shape s;
            tet_shape(d.coords, t, s);
            const int a = local_index(t, u);
            const double c2 = d.c_tet ? d.c_tet[e] * d.c_tet[e] : 1.0;
            for (int b = 0; b < 4; ++b) {
                const double gg = s.g[a][0] * s.g[b][0] + s.g[a][1] * s.g[b][1] + s.g[a][2] * s.g[b][2];
                const int32_t j = hp.iperm[size_t(t[b])];
                const int64_t pos = r0 + (std::lower_bound(c.begin(), c.end(), j) - c.begin());
                hp.k1val[size_t(pos)] += s.vol * gg;
                hp.kval[size_t(pos)] += c2 * (s.vol * gg);
            }
            m += 0.25 * s.vol;
        }
        hp.mass[size_t(i)] = m;
    });
    cols.clear();
    cols.shrink_to_fit();

    // Boundary faces: a face of tetrahedron e is on the boundary when no other
    // tetrahedron holds all three of its nodes.
    static const int kFace[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};
    std::vector<uint8_t> face_on_boundary(size_t(4 * E), 0);
    if (d.absorbing) {
        parallel_for(E, [&](int64_t e) {
            const int32_t *t = d.tets + 4 * e;
            for (int f = 0; f < 4; ++f) {
                const int32_t a = t[kFace[f][0]], b = t[kFace[f][1]], c = t[kFace[f][2]];
                bool shared = false;
                for (int64_t q = inc_ptr[a]; q < inc_ptr[a + 1] && !shared; ++q) {
                    const int64_t o = inc[size_t(q)];
                    if (o == e) continue;
                    const int32_t *u = d.tets + 4 * o;
                    shared = local_index(u, b) >= 0 && local_index(u, c) >= 0;
                }
                face_on_boundary[size_t(4 * e + f)] = shared ? 0 : 1;
            }
        });
    }
    // B_ij = sum over boundary faces F containing i and j of (1/c_e) |F|/12 (1 + delta_ij),
    // the consistent P1 face mass; c_e is the speed of the face's tetrahedron.
    hp.boff.assign(size_t(N), -1);
    hp.n_boundary = 0;
    {
        int64_t off = 0;
        for (int32_t i = 0; i < N; ++i) {
            const int32_t u = hp.perm[size_t(i)];
            bool onb = false;
            for (int64_t q = inc_ptr[u]; q < inc_ptr[u + 1] && !onb; ++q) {
                const int64_t e = inc[size_t(q)];
                const int a = local_index(d.tets + 4 * e, u);
                for (int f = 0; f < 4 && !onb; ++f)
                    if (f != a && face_on_boundary[size_t(4 * e + f)]) onb = true;
            }
            if (onb) {
                hp.boff[i] = int32_t(off);
                off += hp.rowptr[i + 1] - hp.rowptr[i];
                ++hp.n_boundary;
            }
        }
        hp.bval.assign(size_t(off), 0.0);
    }
    parallel_for(N, [&](int64_t i) {
        if (hp.boff[i] < 0) return;
        const int32_t r0 = hp.rowptr[i], r1 = hp.rowptr[i + 1];
        const int32_t u = hp.perm[size_t(i)];
        for (int64_t q = inc_ptr[u]; q < inc_ptr[u + 1]; ++q) {
            const int64_t e = inc[size_t(q)];
            const int32_t *t = d.tets + 4 * e;
            const int a = local_index(t, u);
            for (int f = 0; f < 4; ++f) {
                if (f == a || !face_on_boundary[size_t(4 * e + f)]) continue;
                const double *x0 = d.coords + 3 * int64_t(t[kFace[f][0]]);
                const double *x1 = d.coords + 3 * int64_t(t[kFace[f][1]]);
                const double *x2 = d.coords + 3 * int64_t(t[kFace[f][2]]);
                const double u[3] = {x1[0] - x0[0], x1[1] - x0[1], x1[2] - x0[2]};
                const double v[3] = {x2[0] - x0[0], x2[1] - x0[1], x2[2] - x0[2]};
                const double n[3] = {u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]};
                const double area = 0.5 * std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
                const double scale = (d.c_tet ? 1.0 / d.c_tet[e] : 1.0) * area / 12.0;
                for (int k = 0; k < 3; ++k) {
                    const int32_t j = hp.iperm[size_t(t[kFace[f][k]])];
                    const int32_t *lo = hp.col.data() + r0, *hi = hp.col.data() + r1;
                    const int64_t pos = std::lower_bound(lo, hi, j) - hp.col.data();
                    hp.bval[size_t(hp.boff[i] + (pos - r0))] += (j == int32_t(i) ? 2.0 : 1.0) * scale;
                }
            }
        }
    });
    hp.nnz_b = 0;
    for (double v : hp.bval)
        if (v != 0.0) ++hp.nnz_b;

    // map sensor nodes to the internal numbering
    for (auto &v : hp.snode) v = hp.iperm[size_t(v)];

    // Pi^T as node-major CSR (entries with a zero weight carry nothing and are dropped)
    {
        std::vector<std::array<int64_t, 3>> ent;  // (node, sensor, slot)
        for (int32_t s = 0; s < S; ++s)
            for (int k = 0; k < 4; ++k)
                if (hp.sw[4 * s + k] != 0.0) ent.push_back({hp.snode[4 * s + k], s, k});
        std::sort(ent.begin(), ent.end());
        hp.injptr.assign(size_t(N) + 1, 0);
        for (auto &t : ent) ++hp.injptr[size_t(t[0]) + 1];
        for (int32_t i = 0; i < N; ++i) hp.injptr[i + 1] += hp.injptr[i];
        hp.injs.resize(ent.size());
        hp.injw.resize(ent.size());
        for (size_t q = 0; q < ent.size(); ++q) {
            hp.injs[q] = int32_t(ent[q][1]);
            hp.injw[q] = hp.sw[size_t(4 * ent[q][1] + ent[q][2])];
        }
    }

    build_padded_rows(hp);
    hp.lambda_max = estimate_lambda_max(hp, 150);
    if (d.check_dt) {
        const double x = d.dt * d.dt * 1.02 * hp.lambda_max;
        if (!(x < 4.0)) {
            err = "dt violates the leapfrog CFL bound: dt^2 * lambda_max(M_L^-1 K) = " + std::to_string(x) +
                  " >= 4 (lambda_max ~ " + std::to_string(hp.lambda_max) + ")";
            return PAT_ERR_UNSTABLE_DT;
        }
        if (d.absorbing) {
            const double g = energy_growth(hp, 300);
            if (!(g < 2.0)) {
                err = "explicit absorbing term makes the step unstable at this dt (energy grew by " +
                      std::to_string(g) + " over 300 steps)";
                return PAT_ERR_UNSTABLE_DT;
            }
        }
    }
    return PAT_OK;
}

void build_padded_rows(HostProblem &hp) {
    const int W = HostProblem::kEll;
    const int32_t N = hp.n;
    hp.ell_col.assign(size_t(N) * W, 0);
    hp.ell_val.assign(size_t(N) * W, 0.0);
    hp.xptr.assign(size_t(N) + 1, 0);
    hp.bsoff.assign(size_t(N), -1);
    for (int32_t i = 0; i < N; ++i) {
        const int32_t len = hp.rowptr[i + 1] - hp.rowptr[i];
        hp.xptr[i + 1] = hp.xptr[i] + (len > W ? len - W : 0);
    }
    hp.xcol.assign(size_t(hp.xptr[N]), 0);
    hp.xval.assign(size_t(hp.xptr[N]), 0.0);
    int64_t boff = 0;
    for (int32_t i = 0; i < N; ++i)
        if (hp.boff[i] >= 0) {
            hp.bsoff[i] = int32_t(boff);
            boff += W + (hp.xptr[i + 1] - hp.xptr[i]);
        }
    hp.bslot.assign(size_t(boff), 0.0);
    hp.bnum.assign(size_t(N), 0);
    std::vector<int32_t> order;
    for (int32_t i = 0; i < N; ++i) {
        const int32_t k0 = hp.rowptr[i], len = hp.rowptr[i + 1] - k0;
        // slot order: the diagonal first (the step kernels read the row's own state
        // from that gather), then for boundary rows the other entries with a nonzero B
        // (so the boundary sums touch only bnum[i] slots), then the rest, each group in
        // column order
        order.resize(size_t(len));
        int32_t diag = -1;
        for (int32_t j = 0; j < len; ++j)
            if (hp.col[k0 + j] == i) diag = j;
        const bool bnd = hp.boff[i] >= 0;
        auto has_b = [&](int32_t j) { return bnd && hp.bval[size_t(hp.boff[i] + j)] != 0.0; };
        int32_t o = 0;
        if (diag >= 0) order[size_t(o++)] = diag;
        for (int32_t j = 0; j < len; ++j)
            if (j != diag && has_b(j)) order[size_t(o++)] = j;
        const int32_t nb = bnd ? o : 0;
        for (int32_t j = 0; j < len; ++j)
            if (j != diag && !has_b(j)) order[size_t(o++)] = j;
        hp.bnum[size_t(i)] = nb;
        for (int j = 0; j < W; ++j) {
            hp.ell_col[size_t(i) * W + j] = j < len ? hp.col[k0 + order[size_t(j)]] : i;
            hp.ell_val[size_t(i) * W + j] = j < len ? hp.kval[k0 + order[size_t(j)]] : 0.0;
        }
        for (int32_t j = W; j < len; ++j) {
            hp.xcol[hp.xptr[i] + j - W] = hp.col[k0 + order[size_t(j)]];
            hp.xval[hp.xptr[i] + j - W] = hp.kval[k0 + order[size_t(j)]];
        }
        if (hp.boff[i] >= 0)
            for (int32_t j = 0; j < len; ++j)
                hp.bslot[size_t(hp.bsoff[i] + j)] = hp.bval[size_t(hp.boff[i] + order[size_t(j)])];
    }
}

void build_halo_tiles(const HostProblem &hp, HaloTiles &ht) {
    const int W = HostProblem::kEll;
    const int32_t N = hp.n;
    ht.desc.clear();
    ht.hrow.clear();
    ht.meta.clear();
    auto pad4 = [](size_t k) { return int32_t((k + 3) / 4 * 4); };
    auto is_bnd = [&](int32_t i) { return hp.bsoff[size_t(i)] >= 0; };
    // B slots of boundary row i: the first min(bnum, kEll) padded slots
    auto nbs = [&](int32_t i) { return is_bnd(i) ? std::min(hp.bnum[size_t(i)], W) : 0; };
    std::vector<int32_t> kc, bc, kt, bt;
    int32_t r0 = 0;
    while (r0 < N) {
        kc.clear();
        bc.clear();
        int32_t r1 = r0;
        while (r1 < N && r1 - r0 < HaloTiles::kRows) {
            kt = kc;
            bt = bc;
            for (int j = 0; j < W; ++j) kt.push_back(hp.ell_col[size_t(r1) * W + j]);
            for (int j = 0; j < nbs(r1); ++j) bt.push_back(hp.ell_col[size_t(r1) * W + j]);
            std::sort(kt.begin(), kt.end());
            kt.erase(std::unique(kt.begin(), kt.end()), kt.end());
            std::sort(bt.begin(), bt.end());
            bt.erase(std::unique(bt.begin(), bt.end()), bt.end());
            if (pad4(kt.size()) + pad4(bt.size()) > HaloTiles::kMax) break;
            kc.swap(kt);
            bc.swap(bt);
            ++r1;
        }
        const int32_t nr = r1 - r0, nk4 = pad4(kc.size()), nb4 = pad4(bc.size());
        const int32_t h0 = int32_t(ht.hrow.size());
        for (int32_t k = 0; k < nk4; ++k) ht.hrow.push_back(kc[size_t(std::min<int32_t>(k, int32_t(kc.size()) - 1))]);
        for (int32_t k = 0; k < nb4; ++k) ht.hrow.push_back(bc[size_t(std::min<int32_t>(k, int32_t(bc.size()) - 1))]);
        int32_t nbr = 0;
        for (int32_t i = r0; i < r1; ++i) nbr += is_bnd(i) ? 1 : 0;
        const size_t m0 = ht.meta.size();
        ht.meta.resize(m0 + size_t(nr) * (4 + 4 + 16) + size_t(nbr) * (16 + 4), 0u);
        uint32_t *loc = ht.meta.data() + m0, *info = loc + size_t(nr) * 4, *kv = info + size_t(nr) * 4,
                 *bw = kv + size_t(nr) * 16, *bloc = bw + size_t(nbr) * 16;
        auto fbits = [](double v) {
            const float f = float(v);
            uint32_t u;
            std::memcpy(&u, &f, 4);
            return u;
        };
        int32_t br = 0;
        for (int32_t i = r0; i < r1; ++i) {
            const size_t li = size_t(i - r0);
            const int32_t nx = hp.xptr[size_t(i) + 1] - hp.xptr[size_t(i)];
            const int32_t ninj = hp.injptr[size_t(i) + 1] - hp.injptr[size_t(i)];
            if (hp.bnum[size_t(i)] > 255 || nx > 255 || ninj > 255) {  // a count beyond its byte: no halo tiles
                ht = HaloTiles{};
                return;
            }
            for (int j = 0; j < W; ++j) {
                const int32_t c = hp.ell_col[size_t(i) * W + j];
                const uint32_t kl = uint32_t(std::lower_bound(kc.begin(), kc.end(), c) - kc.begin());
                loc[li * 4 + j / 4] |= kl << (8 * (j % 4));
                kv[li * 16 + j] = fbits(hp.ell_val[size_t(i) * W + j]);
            }
            info[li * 4 + 0] = fbits(hp.dt / hp.mass[size_t(i)]);
            info[li * 4 + 1] = uint32_t(is_bnd(i) ? br : 0xFF) | (uint32_t(hp.bnum[size_t(i)]) << 8) |
                               (uint32_t(nx) << 16) | (uint32_t(ninj) << 24);
            info[li * 4 + 2] = uint32_t(hp.xptr[size_t(i)]);
            info[li * 4 + 3] = uint32_t(hp.injptr[size_t(i)]);
            if (is_bnd(i)) {
                for (int j = 0; j < W; ++j) {
                    bw[size_t(br) * 16 + j] = fbits(hp.bslot[size_t(hp.bsoff[size_t(i)]) + j]);
                    if (j < nbs(i)) {
                        const int32_t c = hp.ell_col[size_t(i) * W + j];
                        const uint32_t bl = uint32_t(std::lower_bound(bc.begin(), bc.end(), c) - bc.begin());
                        bloc[size_t(br) * 4 + j / 4] |= bl << (8 * (j % 4));
                    }
                }
                ++br;
            }
        }
        constexpr int B = HaloTiles::kNrBits;
        const int32_t d[4] = {r0, h0, int32_t(m0 / 4), nr | (nk4 << B) | (nb4 << (B + 8)) | (nbr << (B + 16))};
        ht.desc.insert(ht.desc.end(), d, d + 4);
        r0 = r1;
    }
    ht.n_tiles = int32_t(ht.desc.size() / 4);
}

namespace {
void spmv_host(const HostProblem &hp, const std::vector<double> &val, const std::vector<double> &x,
               std::vector<double> &y) {
    parallel_for(hp.n, [&](int64_t i) {
        double s = 0.0;
        for (int32_t k = hp.rowptr[i]; k < hp.rowptr[i + 1]; ++k) s += val[size_t(k)] * x[size_t(hp.col[k])];
        y[size_t(i)] = s;
    });
}
}  // namespace

double estimate_lambda_max(const HostProblem &hp, int iters) {
    const int32_t N = hp.n;
    std::vector<double> x(N), y(N), z(N);
    for (int32_t i = 0; i < N; ++i) x[i] = ((i & 1) ? -1.0 : 1.0) + 0.25 * std::sin(0.37 * i);
    double lam = 0.0;
    for (int it = 0; it < iters; ++it) {
        double nx = 0.0;
        for (double v : x) nx += v * v;
        nx = std::sqrt(nx);
        for (int32_t i = 0; i < N; ++i) z[i] = x[i] / nx / std::sqrt(hp.mass[i]);
        spmv_host(hp, hp.kval, z, y);
        double rq = 0.0;
        for (int32_t i = 0; i < N; ++i) {
            y[i] /= std::sqrt(hp.mass[i]);
            rq += y[i] * x[i] / nx;
        }
        lam = rq;
        x.swap(y);
    }
    return lam;
}

double energy_growth(const HostProblem &hp, int steps) {
    const int32_t N = hp.n;
    const double dt = hp.dt;
    std::vector<double> P(N), V(N, 0.0), Vn(N), kp(N), kv(N);
    uint64_t st = 0x9E3779B97F4A7C15ull;
    for (int32_t i = 0; i < N; ++i) {
        st = st * 6364136223846793005ull + 1442695040888963407ull;
        P[i] = double(int64_t(st >> 11)) / double(1ull << 53) - 0.5;
    }
    // energy 1/2 v'M v + 1/2 p'K p - dt^2/8 v'K v at integer steps (p = P - dt/2 v)
    auto energy = [&]() {
        std::vector<double> p(N);
        for (int32_t i = 0; i < N; ++i) p[i] = P[i] - 0.5 * dt * V[i];
        spmv_host(hp, hp.kval, p, kp);
        spmv_host(hp, hp.kval, V, kv);
        double e = 0.0;
        for (int32_t i = 0; i < N; ++i)
            e += 0.5 * hp.mass[i] * V[i] * V[i] + 0.5 * p[i] * kp[i] - dt * dt / 8.0 * V[i] * kv[i];
        return e;
    };
    // start from p(0) = random, v(0) = 0 (P = p at step 0)
    const double e0 = energy();
    for (int s = 0; s < steps; ++s) {
        parallel_for(N, [&](int64_t i) {
            double acc = 0.0;
            for (int32_t k = hp.rowptr[i]; k < hp.rowptr[i + 1]; ++k) acc += hp.kval[size_t(k)] * P[size_t(hp.col[k])];
            if (hp.boff[i] >= 0)
                for (int32_t k = hp.rowptr[i]; k < hp.rowptr[i + 1]; ++k)
                    acc += hp.bval[size_t(hp.boff[i] + k - hp.rowptr[i])] * V[size_t(hp.col[k])];
            Vn[size_t(i)] = V[size_t(i)] - dt / hp.mass[i] * acc;
        });
        for (int32_t i = 0; i < N; ++i) P[i] += dt * Vn[i];
        V.swap(Vn);
    }
    const double e1 = energy();
    return std::isfinite(e1) ? e1 / e0 : std::numeric_limits<double>::infinity();
}

}  // namespace pat
