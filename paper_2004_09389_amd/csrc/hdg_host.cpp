// Host-side setup pieces: mesh topology, reference-element tables, P1 level
// operators and the dense coarsest-level inverse.
#include <algorithm>
#include <cmath>
#include <map>
#include <unordered_map>

#include "hdg_host.h"

namespace hdg {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

}  // namespace hdg

extern "C" const char *hdg_last_error(void) { return hdg::g_last_error.c_str(); }

namespace hdg {

// ------------------------------------------------------------------ topology
//
// Skeleton of a closed (periodic or spherical) triangulation: every facet is
// the side of exactly two cells (spatial discretisation section).  A facet is
// identified by its two end vertices and the periodic offset between them, so
// meshes whose cells share more than one facet through the periodic wrap
// (down to the 1 x 1 square: 2 cells, 3 facets, 1 vertex) are handled.

namespace {
struct EdgeKey {
    int32_t va, vb, dx, dy;
    bool operator==(const EdgeKey &o) const {
        return va == o.va && vb == o.vb && dx == o.dx && dy == o.dy;
    }
};
struct EdgeHash {
    size_t operator()(const EdgeKey &k) const {
        uint64_t h = (uint64_t)(uint32_t)k.va * 0x9E3779B97F4A7C15ull;
        h ^= (uint64_t)(uint32_t)k.vb + 0x632BE59BD9B4E019ull + (h << 6) + (h >> 2);
        h ^= (uint64_t)(uint32_t)(k.dx * 1024 + k.dy) + 0x85EBCA77C2B2AE63ull + (h << 6) + (h >> 2);
        return (size_t)h;
    }
};

EdgeKey make_key(int va, const int *sa, int vb, const int *sb) {
    int dx = sb[0] - sa[0], dy = sb[1] - sa[1];
    if (va < vb) return {va, vb, dx, dy};
    if (va > vb) return {vb, va, -dx, -dy};
    // same vertex at both ends (periodic wrap): orientation-free offset
    if (dx < 0 || (dx == 0 && dy < 0)) { dx = -dx; dy = -dy; }
    return {va, va, dx, dy};
}
}  // namespace

Topology build_topology(const hdg_mesh &mesh) {
    Topology t;
    const int nk = mesh.n_cell;
    t.n_cell = nk;
    t.cell_facet.assign((size_t)nk * 3, -1);
    t.cell_rev.assign((size_t)nk * 3, 0);
    std::unordered_map<EdgeKey, int, EdgeHash> seen;
    seen.reserve((size_t)nk * 2);
    static const int zero[2] = {0, 0};
    for (int K = 0; K < nk; ++K) {
        for (int i = 0; i < 3; ++i) {
            int a = (i + 1) % 3, b = (i + 2) % 3;
            int va = mesh.cell_vert[3 * K + a], vb = mesh.cell_vert[3 * K + b];
            HDG_REQUIRE(va >= 0 && va < mesh.n_vert && vb >= 0 && vb < mesh.n_vert,
                        "cell_vert holds an out-of-range vertex id");
            const int *sa = mesh.cell_shift ? mesh.cell_shift + 6 * K + 2 * a : zero;
            const int *sb = mesh.cell_shift ? mesh.cell_shift + 6 * K + 2 * b : zero;
            EdgeKey key = make_key(va, sa, vb, sb);
            auto it = seen.find(key);
            if (it == seen.end()) {
                int e = t.n_facet++;
                seen.emplace(key, e);
                t.facet_cell.push_back(K);
                t.facet_cell.push_back(-1);
                t.facet_loc.push_back(i);
                t.facet_loc.push_back(-1);
                t.facet_vert.push_back(va);
                t.facet_vert.push_back(vb);
                t.cell_facet[3 * K + i] = e;
            } else {
                int e = it->second;
                HDG_REQUIRE(t.facet_cell[2 * e + 1] < 0, "a facet is shared by more than two cells");
                t.facet_cell[2 * e + 1] = K;
                t.facet_loc[2 * e + 1] = i;
                t.cell_facet[3 * K + i] = e;
                t.cell_rev[3 * K + i] = 1;
            }
        }
    }
    for (int e = 0; e < t.n_facet; ++e)
        HDG_REQUIRE(t.facet_cell[2 * e + 1] >= 0, "boundary facet: the mesh must be closed or periodic");
    return t;
}

std::vector<double> cell_corners(const hdg_mesh &mesh) {
    std::vector<double> x((size_t)mesh.n_cell * 9);
    for (int K = 0; K < mesh.n_cell; ++K)
        for (int k = 0; k < 3; ++k) {
            int v = mesh.cell_vert[3 * K + k];
            for (int d = 0; d < 3; ++d) x[9 * K + 3 * k + d] = mesh.vert_xyz[3 * v + d];
            if (mesh.geom == HDG_TORUS && mesh.cell_shift) {
                x[9 * K + 3 * k + 0] += mesh.period * mesh.cell_shift[6 * K + 2 * k + 0];
                x[9 * K + 3 * k + 1] += mesh.period * mesh.cell_shift[6 * K + 2 * k + 1];
            }
        }
    return x;
}

// ------------------------------------------------------------------ reference tables

// Gauss-Legendre points and weights on [0, 1] (Newton iteration on the
// Legendre three-term recurrence).
static void gauss_legendre01(int n, std::vector<double> &x, std::vector<double> &w) {
    x.resize(n);
    w.resize(n);
    for (int i = 0; i < n; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p1 = z; p0 = 1.0; }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        // recompute derivative at the converged root
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; ++k) {
            double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        if (n == 1) { p1 = z; p0 = 1.0; }
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        x[n - 1 - i] = 0.5 * (z + 1.0);
        w[n - 1 - i] = 1.0 / ((1.0 - z * z) * dp * dp);  // = 0.5 * 2/((1-z^2) P'^2)
    }
}

bool invert_dense(std::vector<double> &a, int n) {
    // Gauss-Jordan with partial pivoting, in place
    std::vector<int> piv(n);
    std::vector<double> inv((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) inv[(size_t)i * n + i] = 1.0;
    for (int k = 0; k < n; ++k) {
        int p = k;
        for (int i = k + 1; i < n; ++i)
            if (std::fabs(a[(size_t)i * n + k]) > std::fabs(a[(size_t)p * n + k])) p = i;
        if (std::fabs(a[(size_t)p * n + k]) < 1e-300) return false;
        if (p != k)
            for (int j = 0; j < n; ++j) {
                std::swap(a[(size_t)k * n + j], a[(size_t)p * n + j]);
                std::swap(inv[(size_t)k * n + j], inv[(size_t)p * n + j]);
            }
        double d = 1.0 / a[(size_t)k * n + k];
        for (int j = 0; j < n; ++j) {
            a[(size_t)k * n + j] *= d;
            inv[(size_t)k * n + j] *= d;
        }
        for (int i = 0; i < n; ++i) {
            if (i == k) continue;
            double f = a[(size_t)i * n + k];
            if (f == 0.0) continue;
            for (int j = 0; j < n; ++j) {
                a[(size_t)i * n + j] -= f * a[(size_t)k * n + j];
                inv[(size_t)i * n + j] -= f * inv[(size_t)k * n + j];
            }
        }
    }
    a.swap(inv);
    return true;
}

RefTables build_ref_tables(int p) {
    RefTables R;
    R.p = p;
    const int n = (p + 1) * (p + 2) / 2, m = p + 1;
    R.n = n;
    R.m = m;
    // lattice nodes, j-major then i
    std::vector<double> nx, ny;
    for (int j = 0; j <= p; ++j)
        for (int i = 0; i <= p - j; ++i) {
            nx.push_back((double)i / p);
            ny.push_back((double)j / p);
        }
    // monomials xi^a eta^b, a + b <= p
    std::vector<std::pair<int, int>> ex;
    for (int d = 0; d <= p; ++d)
        for (int a = 0; a <= d; ++a) ex.push_back({a, d - a});
    std::vector<double> V((size_t)n * n);
    for (int k = 0; k < n; ++k)
        for (int al = 0; al < n; ++al)
            V[(size_t)k * n + al] = std::pow(nx[k], ex[al].first) * std::pow(ny[k], ex[al].second);
    if (!invert_dense(V, n)) throw Error{HDG_EINVAL, "singular reference Vandermonde matrix"};
    // V now holds coefficients C[al][i]
    auto eval = [&](double x, double y, double *val, double *dx, double *dy) {
        for (int i = 0; i < n; ++i) {
            double v = 0, gx = 0, gy = 0;
            for (int al = 0; al < n; ++al) {
                int a = ex[al].first, b = ex[al].second;
                double c = V[(size_t)al * n + i];
                v += c * std::pow(x, a) * std::pow(y, b);
                if (a > 0) gx += c * a * std::pow(x, a - 1) * std::pow(y, b);
                if (b > 0) gy += c * b * std::pow(x, a) * std::pow(y, b - 1);
            }
            val[i] = v;
            if (dx) dx[i] = gx;
            if (dy) dy[i] = gy;
        }
    };
    // collapsed Gauss rule with p+3 points per direction (exact to degree 2p+3)
    std::vector<double> gs, gw;
    gauss_legendre01(p + 3, gs, gw);
    R.nq = (p + 3) * (p + 3);
    for (int a = 0; a < p + 3; ++a)
        for (int b = 0; b < p + 3; ++b) {
            double s = gs[a], t = gs[b];
            R.qx.push_back(s * (1.0 - t));
            R.qx.push_back(t);
            R.qw.push_back(gw[a] * gw[b] * (1.0 - t));
        }
    R.M.assign((size_t)n * n, 0.0);
    R.G.assign((size_t)2 * n * n, 0.0);
    R.Phi.assign((size_t)R.nq * n, 0.0);
    std::vector<double> v(n), gx(n), gy(n);
    for (int q = 0; q < R.nq; ++q) {
        eval(R.qx[2 * q], R.qx[2 * q + 1], v.data(), gx.data(), gy.data());
        double w = R.qw[q];
        for (int i = 0; i < n; ++i) {
            R.Phi[(size_t)q * n + i] = v[i];
            for (int j = 0; j < n; ++j) {
                R.M[(size_t)i * n + j] += w * v[i] * v[j];
                R.G[(size_t)i * n + j] += w * v[i] * gx[j];
                R.G[(size_t)n * n + (size_t)i * n + j] += w * v[i] * gy[j];
            }
        }
    }
    // facets: local facet f runs from reference vertex (f+1)%3 to (f+2)%3
    const double vx[3] = {0.0, 1.0, 0.0}, vy[3] = {0.0, 0.0, 1.0};
    std::vector<double> fs, fw;
    gauss_legendre01(p + 2, fs, fw);
    R.E.assign((size_t)3 * n * n, 0.0);
    R.T.assign((size_t)3 * n * m, 0.0);
    R.F.assign((size_t)m * m, 0.0);
    auto mu = [&](double s, double *out) {
        for (int k = 0; k < m; ++k) {
            double r = 1.0;
            for (int l = 0; l < m; ++l)
                if (l != k) r *= (s - (double)l / p) / ((double)k / p - (double)l / p);
            out[k] = r;
        }
    };
    std::vector<double> muv(m);
    for (int f = 0; f < 3; ++f) {
        int a = (f + 1) % 3, b = (f + 2) % 3;
        for (size_t q = 0; q < fs.size(); ++q) {
            double s = fs[q], w = fw[q];
            eval(vx[a] + s * (vx[b] - vx[a]), vy[a] + s * (vy[b] - vy[a]), v.data(), nullptr, nullptr);
            mu(s, muv.data());
            for (int i = 0; i < n; ++i) {
                for (int j = 0; j < n; ++j) R.E[(size_t)f * n * n + (size_t)i * n + j] += w * v[i] * v[j];
                for (int k = 0; k < m; ++k) R.T[(size_t)f * n * m + (size_t)i * m + k] += w * v[i] * muv[k];
            }
            if (f == 0)
                for (int k = 0; k < m; ++k)
                    for (int l = 0; l < m; ++l) R.F[(size_t)k * m + l] += w * muv[k] * muv[l];
        }
    }
    return R;
}

// ------------------------------------------------------------------ P1 levels
//
// Coarse form of the upwind case (Eq. coarse_problem_upwind) scaled to the
// trace system: S_c = (1/kappa) (M_1 + kappa^2 K_1), assembled from the
// closed-form P1 element matrices of each flat cell (mass |K|/12 (1 + d_ij),
// stiffness (e_i . e_j) / (4 |K|) with e_i the edge opposite corner i).

P1Host assemble_p1(const hdg_mesh &mesh, double kappa) {
    P1Host P;
    const int nv = mesh.n_vert;
    P.n = nv;
    std::vector<double> x = cell_corners(mesh);
    std::vector<std::map<int, double>> rows(nv);
    std::vector<double> diag(nv, 0.0);
    for (int K = 0; K < mesh.n_cell; ++K) {
        const double *c = &x[9 * K];
        double e[3][3];
        for (int i = 0; i < 3; ++i)
            for (int d = 0; d < 3; ++d) e[i][d] = c[3 * ((i + 2) % 3) + d] - c[3 * ((i + 1) % 3) + d];
        double ab[3], ac[3], cr[3];
        for (int d = 0; d < 3; ++d) {
            ab[d] = c[3 + d] - c[d];
            ac[d] = c[6 + d] - c[d];
        }
        cr[0] = ab[1] * ac[2] - ab[2] * ac[1];
        cr[1] = ab[2] * ac[0] - ab[0] * ac[2];
        cr[2] = ab[0] * ac[1] - ab[1] * ac[0];
        double area = 0.5 * std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                double kij = (e[i][0] * e[j][0] + e[i][1] * e[j][1] + e[i][2] * e[j][2]) / (4.0 * area);
                double mij = area / 12.0 * (i == j ? 2.0 : 1.0);
                double v = (mij + kappa * kappa * kij) / kappa;
                int vi = mesh.cell_vert[3 * K + i], vj = mesh.cell_vert[3 * K + j];
                if (vi == vj)
                    diag[vi] += v;
                else
                    rows[vi][vj] += v;
            }
    }
    P.rowptr.assign(nv + 1, 0);
    for (int v = 0; v < nv; ++v) P.rowptr[v + 1] = P.rowptr[v] + (int)rows[v].size();
    P.col.reserve(P.rowptr[nv]);
    P.val.reserve(P.rowptr[nv]);
    for (int v = 0; v < nv; ++v)
        for (auto &kv : rows[v]) {
            P.col.push_back(kv.first);
            P.val.push_back(kv.second);
        }
    P.diag = diag;
    return P;
}

// Galerkin coarse form on the finest P1 level, S_c = pi^T S pi (the coarse form
// footnoted in the non-nested multigrid section), from the facet rows of S:
// rows [component / 2][n_facet][2] with component (j m + a) m + k for block j
// (0 = the facet itself, 1..4 = nbr[j - 1]); pi puts (1 - k/p, k/p) of the
// facet's (start, end) vertex values on trace node k.
P1Host galerkin_from_rows(int ne, int m, int nv, const std::vector<double> &rows, const std::vector<int32_t> &nbr,
                          const std::vector<int32_t> &facet_vert) {
    const int p = m - 1;
    std::vector<std::map<int, double>> A(nv);
    for (int e = 0; e < ne; ++e) {
        int id[5] = {e, nbr[e], nbr[(size_t)ne + e], nbr[2 * (size_t)ne + e], nbr[3 * (size_t)ne + e]};
        const int rv[2] = {facet_vert[2 * e], facet_vert[2 * e + 1]};
        for (int j = 0; j < 5; ++j) {
            const int cv[2] = {facet_vert[2 * id[j]], facet_vert[2 * id[j] + 1]};
            for (int a = 0; a < m; ++a)
                for (int k = 0; k < m; ++k) {
                    const int comp = (j * m + a) * m + k;
                    const double sv = rows[((size_t)(comp / 2) * ne + e) * 2 + comp % 2];
                    const double wa[2] = {1.0 - (double)a / p, (double)a / p};
                    const double wk[2] = {1.0 - (double)k / p, (double)k / p};
                    for (int x = 0; x < 2; ++x)
                        for (int y = 0; y < 2; ++y) A[rv[x]][cv[y]] += wa[x] * sv * wk[y];
                }
        }
    }
    P1Host P;
    P.n = nv;
    P.rowptr.assign(nv + 1, 0);
    P.diag.assign(nv, 0.0);
    for (int v = 0; v < nv; ++v) {
        for (auto &kv : A[v]) {
            if (kv.first == v) {
                P.diag[v] = kv.second;
            } else {
                P.col.push_back(kv.first);
                P.val.push_back(kv.second);
            }
        }
        P.rowptr[v + 1] = (int)P.col.size();
    }
    return P;
}

// A_c = P^T A P with P the linear interpolation of the parent map (fine vertex v
// takes half of each of its two parents; an inherited vertex lists one parent twice)
P1Host galerkin_coarsen(const P1Host &F, const int32_t *parents, int nc) {
    std::vector<std::map<int, double>> A(nc);
    auto add_row = [&](int v, int w, double a) {
        for (int x = 0; x < 2; ++x)
            for (int y = 0; y < 2; ++y) A[parents[2 * v + x]][parents[2 * w + y]] += 0.25 * a;
    };
    for (int v = 0; v < F.n; ++v) {
        add_row(v, v, F.diag[v]);
        for (int q = F.rowptr[v]; q < F.rowptr[v + 1]; ++q) add_row(v, F.col[q], F.val[q]);
    }
    P1Host P;
    P.n = nc;
    P.rowptr.assign(nc + 1, 0);
    P.diag.assign(nc, 0.0);
    for (int v = 0; v < nc; ++v) {
        for (auto &kv : A[v]) {
            if (kv.first == v) {
                P.diag[v] = kv.second;
            } else {
                P.col.push_back(kv.first);
                P.val.push_back(kv.second);
            }
        }
        P.rowptr[v + 1] = (int)P.col.size();
    }
    return P;
}

bool spd_inverse(std::vector<double> &a, int n) {
    for (int i = 0; i < n; ++i)
        if (!(a[(size_t)i * n + i] > 0.0)) return false;
    return invert_dense(a, n);
}

}  // namespace hdg

// ------------------------------------------------------------------ the P1 V-cycle as a matrix
//
// One P1 multigrid V-cycle (damped Jacobi with nu sweeps before and after,
// linear-interpolation transfers from the parent pairs, exact solve on level
// 0) is a fixed linear map b -> x on the finest level.  For a small hierarchy
// its matrix is formed once, column by column, and the persistent solve
// applies it as one dense product.
namespace {
struct P1Cycle {
    const std::vector<hdg::P1Host> &ops;
    const int32_t *const *parents;
    const std::vector<double> &ainv;
    int nu;
    double w;

    std::vector<double> ax(int l, const std::vector<double> &x) const {
        const hdg::P1Host &A = ops[l];
        std::vector<double> y(A.n);
        for (int v = 0; v < A.n; ++v) {
            double s = A.diag[v] * x[v];
            for (int k = A.rowptr[v]; k < A.rowptr[v + 1]; ++k) s += A.val[k] * x[A.col[k]];
            y[v] = s;
        }
        return y;
    }
    std::vector<double> cycle(int l, const std::vector<double> &b) const {
        const hdg::P1Host &A = ops[l];
        const int n = A.n;
        std::vector<double> x(n, 0.0);
        if (l == 0) {
            for (int i = 0; i < n; ++i) {
                double s = 0.0;
                for (int j = 0; j < n; ++j) s += ainv[(size_t)i * n + j] * b[j];
                x[i] = s;
            }
            return x;
        }
        for (int v = 0; v < n; ++v) x[v] = w * b[v] / A.diag[v];
        for (int k = 1; k < nu; ++k) {
            const std::vector<double> y = ax(l, x);
            for (int v = 0; v < n; ++v) x[v] += w * (b[v] - y[v]) / A.diag[v];
        }
        std::vector<double> r = ax(l, x);
        for (int v = 0; v < n; ++v) r[v] = b[v] - r[v];
        const int nc = ops[l - 1].n;
        const int32_t *par = parents[l];
        std::vector<double> bc(nc, 0.0);
        for (int v = 0; v < n; ++v)
            for (int k = 0; k < 2; ++k) bc[par[2 * v + k]] += 0.5 * r[v];
        const std::vector<double> xc = cycle(l - 1, bc);
        for (int v = 0; v < n; ++v) x[v] += 0.5 * (xc[par[2 * v]] + xc[par[2 * v + 1]]);
        for (int k = 0; k < nu; ++k) {
            const std::vector<double> y = ax(l, x);
            for (int v = 0; v < n; ++v) x[v] += w * (b[v] - y[v]) / A.diag[v];
        }
        return x;
    }
};
}  // namespace

std::vector<double> hdg::p1_vcycle_matrix(const std::vector<hdg::P1Host> &ops, const int32_t *const *parents, int nu,
                                          double omega) {
    const int n0 = ops[0].n;
    std::vector<double> ainv((size_t)n0 * n0, 0.0);
    for (int v = 0; v < n0; ++v) {
        ainv[(size_t)v * n0 + v] = ops[0].diag[v];
        for (int k = ops[0].rowptr[v]; k < ops[0].rowptr[v + 1]; ++k) ainv[(size_t)v * n0 + ops[0].col[k]] += ops[0].val[k];
    }
    if (!hdg::spd_inverse(ainv, n0)) throw hdg::Error{HDG_EINVAL, "coarsest P1 operator is singular"};
    const P1Cycle cyc{ops, parents, ainv, nu, omega};
    const int top = (int)ops.size() - 1, n = ops[top].n;
    std::vector<double> B((size_t)n * n);
    std::vector<double> e(n, 0.0);
    for (int j = 0; j < n; ++j) {
        e[j] = 1.0;
        const std::vector<double> col = cyc.cycle(top, e);
        e[j] = 0.0;
        for (int i = 0; i < n; ++i) B[(size_t)i * n + j] = col[i];
    }
    return B;
}
