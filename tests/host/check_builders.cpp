// Checks of the host-side builders (mesh topology, reference tables, P1 and
// RT0 coarse levels) against properties the mathematics fixes, meant to be
// compiled with the host compiler alone under the address and
// undefined-behaviour sanitizers.  Test infrastructure: it links the
// library's host sources directly and touches no GPU.
//
// Usage: check_builders <hierarchy file>...   (format written by the test:
//   int32 n_levels, then per level int32 geom, n_vert, n_cell, float64 period,
//   float64 vert[n_vert][3], int32 cell_vert[n_cell][3], int32 shift[n_cell][3][2],
//   then per level above the coarsest int32 parents[n_vert][2])
// Prints one "ok <check>" line per check; exits 1 at the first failure.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "../../paper_2004_09389_amd/csrc/hdg_host.h"

namespace {

struct Level {
    int geom = 0, nv = 0, nk = 0;
    double period = 1.0;
    std::vector<double> xyz;
    std::vector<int32_t> cv, sh, par;
    hdg_mesh mesh() const { return hdg_mesh{geom, nv, nk, period, xyz.data(), cv.data(), sh.data()}; }
};

[[noreturn]] void fail(const std::string &what) {
    std::printf("FAIL %s\n", what.c_str());
    std::fflush(stdout);
    std::exit(1);
}
void ok(const std::string &what) { std::printf("ok %s\n", what.c_str()); }
void require(bool c, const std::string &what) {
    if (!c) fail(what);
}

template <typename T>
void read_into(FILE *f, std::vector<T> &v, size_t n) {
    v.resize(n);
    if (n && std::fread(v.data(), sizeof(T), n, f) != n) fail("short read");
}

std::vector<Level> read_hierarchy(const char *path) {
    FILE *f = std::fopen(path, "rb");
    if (!f) fail(std::string("cannot open ") + path);
    int32_t nl = 0;
    if (std::fread(&nl, 4, 1, f) != 1 || nl < 1 || nl > 16) fail("bad header");
    std::vector<Level> L(nl);
    for (auto &l : L) {
        int32_t h[3];
        if (std::fread(h, 4, 3, f) != 3 || std::fread(&l.period, 8, 1, f) != 1) fail("bad level header");
        l.geom = h[0];
        l.nv = h[1];
        l.nk = h[2];
        read_into(f, l.xyz, (size_t)3 * l.nv);
        read_into(f, l.cv, (size_t)3 * l.nk);
        read_into(f, l.sh, (size_t)6 * l.nk);
    }
    for (int i = 1; i < nl; ++i) read_into(f, L[i].par, (size_t)2 * L[i].nv);
    std::fclose(f);
    return L;
}

double max_abs(const std::vector<double> &a) {
    double m = 0.0;
    for (double v : a) m = std::fmax(m, std::fabs(v));
    return m;
}

// dense [n][n] of a P1 operator
std::vector<double> dense_p1(const hdg::P1Host &A) {
    std::vector<double> D((size_t)A.n * A.n, 0.0);
    for (int v = 0; v < A.n; ++v) {
        D[(size_t)v * A.n + v] += A.diag[v];
        for (int k = A.rowptr[v]; k < A.rowptr[v + 1]; ++k) D[(size_t)v * A.n + A.col[k]] += A.val[k];
    }
    return D;
}

std::vector<double> matmul(const std::vector<double> &A, const std::vector<double> &B, int n, int k, int m) {
    std::vector<double> C((size_t)n * m, 0.0);
    for (int i = 0; i < n; ++i)
        for (int q = 0; q < k; ++q) {
            const double a = A[(size_t)i * k + q];
            if (a != 0.0)
                for (int j = 0; j < m; ++j) C[(size_t)i * m + j] += a * B[(size_t)q * m + j];
        }
    return C;
}
std::vector<double> transpose(const std::vector<double> &A, int n, int m) {
    std::vector<double> T((size_t)m * n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < m; ++j) T[(size_t)j * n + i] = A[(size_t)i * m + j];
    return T;
}
double sym_defect(const std::vector<double> &A, int n) {
    double d = 0.0;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) d = std::fmax(d, std::fabs(A[(size_t)i * n + j] - A[(size_t)j * n + i]));
    return d / std::fmax(max_abs(A), 1e-300);
}
// true when the symmetric matrix is positive definite (Cholesky succeeds)
bool cholesky_ok(std::vector<double> A, int n) {
    for (int j = 0; j < n; ++j) {
        double d = A[(size_t)j * n + j];
        for (int k = 0; k < j; ++k) d -= A[(size_t)j * n + k] * A[(size_t)j * n + k];
        if (!(d > 0.0)) return false;
        d = std::sqrt(d);
        A[(size_t)j * n + j] = d;
        for (int i = j + 1; i < n; ++i) {
            double s = A[(size_t)i * n + j];
            for (int k = 0; k < j; ++k) s -= A[(size_t)i * n + k] * A[(size_t)j * n + k];
            A[(size_t)i * n + j] = s / d;
        }
    }
    return true;
}
double identity_defect(const std::vector<double> &A, int n) {
    double d = 0.0;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) d = std::fmax(d, std::fabs(A[(size_t)i * n + j] - (i == j ? 1.0 : 0.0)));
    return d;
}

double total_area(const hdg_mesh &m) {
    const std::vector<double> x = hdg::cell_corners(m);
    double s = 0.0;
    for (int K = 0; K < m.n_cell; ++K) {
        const double *c = &x[9 * (size_t)K];
        const double a[3] = {c[3] - c[0], c[4] - c[1], c[5] - c[2]}, b[3] = {c[6] - c[0], c[7] - c[1], c[8] - c[2]};
        const double cr[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
        s += 0.5 * std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
    }
    return s;
}

// interpolation matrix [n_fine][n_coarse] of a parent map (half of each parent)
std::vector<double> p1_prolongation(const std::vector<int32_t> &par, int nf, int nc) {
    std::vector<double> P((size_t)nf * nc, 0.0);
    for (int v = 0; v < nf; ++v)
        for (int k = 0; k < 2; ++k) P[(size_t)v * nc + par[2 * v + k]] += 0.5;
    return P;
}

void check_topology(const std::string &tag, const Level &L) {
    const hdg_mesh m = L.mesh();
    const hdg::Topology t = hdg::build_topology(m);
    require(2 * t.n_facet == 3 * t.n_cell, tag + " topology: 2 facets per 3 cells");
    for (int e = 0; e < t.n_facet; ++e)
        for (int s = 0; s < 2; ++s) {
            const int K = t.facet_cell[2 * e + s], i = t.facet_loc[2 * e + s];
            require(K >= 0 && K < t.n_cell && i >= 0 && i < 3, tag + " topology: facet side in range");
            require(t.cell_facet[3 * K + i] == e, tag + " topology: cell_facet inverts facet_cell");
            require(t.cell_rev[3 * K + i] == s, tag + " topology: the second side runs against the facet");
        }
    // Euler characteristic: 2 on the sphere, 0 on the torus
    const int chi = L.nv - t.n_facet + t.n_cell;
    require(chi == (L.geom == HDG_SPHERE ? 2 : 0), tag + " topology: Euler characteristic");
    ok(tag + " topology");
}

void check_ref_tables() {
    for (int p = 1; p <= 3; ++p) {
        const hdg::RefTables R = hdg::build_ref_tables(p);
        const std::string tag = "ref tables p=" + std::to_string(p);
        double sw = 0.0, sm = 0.0, sf = 0.0;
        for (double w : R.qw) sw += w;
        for (double v : R.M) sm += v;
        for (double v : R.F) sf += v;
        require(std::fabs(sw - 0.5) < 1e-14, tag + ": quadrature weights sum to the area 1/2");
        require(std::fabs(sm - 0.5) < 1e-13, tag + ": mass entries sum to the area");
        require(std::fabs(sf - 1.0) < 1e-13, tag + ": facet mass entries sum to the length");
        for (int q = 0; q < R.nq; ++q) {
            double s = 0.0;
            for (int i = 0; i < R.n; ++i) s += R.Phi[(size_t)q * R.n + i];
            require(std::fabs(s - 1.0) < 1e-12, tag + ": basis is a partition of unity");
        }
        // int phi_i d_r phi_j summed over j is zero (the basis sums to a constant)
        for (int d = 0; d < 2; ++d)
            for (int i = 0; i < R.n; ++i) {
                double s = 0.0;
                for (int j = 0; j < R.n; ++j) s += R.G[((size_t)d * R.n + i) * R.n + j];
                require(std::fabs(s) < 1e-12, tag + ": derivative of the constant vanishes");
            }
        ok(tag);
    }
}

void check_p1(const std::string &tag, const std::vector<Level> &H, double kappa) {
    std::vector<hdg::P1Host> ops;
    for (const Level &L : H) ops.push_back(hdg::assemble_p1(L.mesh(), kappa));
    for (size_t l = 0; l < H.size(); ++l) {
        const hdg::P1Host &A = ops[l];
        const std::vector<double> D = dense_p1(A);
        require(sym_defect(D, A.n) < 1e-14, tag + " P1: symmetric");
        double s = 0.0;
        for (double v : D) s += v;   // 1^T (M + kappa^2 K) 1 / kappa = area / kappa
        const double area = total_area(H[l].mesh());
        require(std::fabs(s - area / kappa) < 1e-12 * area / kappa, tag + " P1: constants see only the mass");
        require(cholesky_ok(D, A.n), tag + " P1: positive definite");
        if (A.n <= 200) {
            std::vector<double> inv = D;
            require(hdg::spd_inverse(inv, A.n), tag + " P1: spd_inverse succeeds");
            require(identity_defect(matmul(D, inv, A.n, A.n, A.n), A.n) < 1e-10, tag + " P1: A A^-1 = I");
        }
    }
    // Galerkin coarsening equals P^T A P with the parent interpolation; on the
    // flat nested torus it equals the coarse discretisation itself
    for (size_t l = 1; l < H.size(); ++l) {
        const int nf = H[l].nv, nc = H[l - 1].nv;
        const hdg::P1Host G = hdg::galerkin_coarsen(ops[l], H[l].par.data(), nc);
        const std::vector<double> P = p1_prolongation(H[l].par, nf, nc);
        const std::vector<double> PtAP = matmul(transpose(P, nf, nc), matmul(dense_p1(ops[l]), P, nf, nf, nc), nc, nf, nc);
        const std::vector<double> Gd = dense_p1(G);
        double d = 0.0;
        for (size_t i = 0; i < Gd.size(); ++i) d = std::fmax(d, std::fabs(Gd[i] - PtAP[i]));
        require(d < 1e-12 * max_abs(PtAP), tag + " P1: Galerkin coarsening is P^T A P");
        if (H[l].geom == HDG_TORUS) {
            const std::vector<double> Cd = dense_p1(ops[l - 1]);
            double e = 0.0;
            for (size_t i = 0; i < Cd.size(); ++i) e = std::fmax(e, std::fabs(Gd[i] - Cd[i]));
            require(e < 1e-12 * max_abs(Cd), tag + " P1: nested flat levels: Galerkin = rediscretised");
        }
    }
    // V-cycle matrix: one level is the exact inverse; several levels give a
    // symmetric, convergent cycle (spectral radius of I - B A below one)
    {
        std::vector<hdg::P1Host> one{ops[0]};
        const int32_t *none[1] = {nullptr};
        const int n = ops[0].n;
        const std::vector<double> B = hdg::p1_vcycle_matrix(one, none, 2, 0.6);
        require(identity_defect(matmul(dense_p1(ops[0]), B, n, n, n), n) < 1e-10, tag + " V-cycle: one level is A^-1");
    }
    if (H.size() > 1 && H.back().nv <= 300) {
        std::vector<const int32_t *> par(H.size(), nullptr);
        for (size_t l = 1; l < H.size(); ++l) par[l] = H[l].par.data();
        const int n = ops.back().n;
        const std::vector<double> B = hdg::p1_vcycle_matrix(ops, par.data(), 2, 0.6);
        require(sym_defect(B, n) < 1e-12, tag + " V-cycle: symmetric");
        std::vector<double> E = matmul(B, dense_p1(ops.back()), n, n, n);
        for (size_t i = 0; i < E.size(); ++i) E[i] = (i % (n + 1) == 0 ? 1.0 : 0.0) - E[i];
        std::vector<double> x(n);
        for (int i = 0; i < n; ++i) x[i] = std::sin(1.0 + 3.7 * i);
        double rho = 0.0;
        for (int it = 0; it < 60; ++it) {
            std::vector<double> y = matmul(E, x, n, n, 1);
            double a = 0.0, b = 0.0;
            for (int i = 0; i < n; ++i) {
                a += y[i] * y[i];
                b += x[i] * x[i];
            }
            rho = std::sqrt(a / b);
            for (int i = 0; i < n; ++i) x[i] = y[i] / std::sqrt(a);
        }
        require(rho < 0.9, tag + " V-cycle: convergent");
    }
    ok(tag + " P1 levels");
}

void check_rt0(const std::string &tag, const std::vector<Level> &H, double kappa) {
    std::vector<hdg::Rt0Host> R;
    for (const Level &L : H) R.push_back(hdg::build_rt0_level(L.mesh(), kappa, true));
    for (size_t l = 0; l < H.size(); ++l) {
        const hdg::Rt0Host &L = R[l];
        const int ne = L.ne, nv = L.nv;
        const std::vector<double> D = hdg::rt0_dense(L);
        require(sym_defect(D, ne) < 1e-13, tag + " RT0: symmetric");
        require(cholesky_ok(D, ne), tag + " RT0: positive definite");
        for (int v = 0; v < nv; ++v) {   // patch inverses invert the patch blocks of S_c
            int np = 0;
            while (np < hdg::RT_PV && L.pf[(size_t)np * nv + v] >= 0) ++np;
            require(np >= 1, tag + " RT0: every vertex has a patch");
            for (int a = 0; a < np; ++a)
                for (int b = 0; b < np; ++b) {
                    double s = 0.0;
                    for (int c = 0; c < np; ++c)
                        s += L.pinv[(size_t)(a * hdg::RT_PV + c) * nv + v] *
                             D[(size_t)L.pf[(size_t)c * nv + v] * ne + L.pf[(size_t)b * nv + v]];
                    require(std::fabs(s - (a == b ? 1.0 : 0.0)) < 1e-10, tag + " RT0: patch inverse");
                }
        }
        // the Lax-Friedrichs prolongation reproduces a constant vector field
        // from its RT0 interpolant (RT0 contains the constants)
        const hdg_mesh m = H[l].mesh();
        const std::vector<double> corners = hdg::cell_corners(m);
        for (int p = 1; p <= 3; ++p) {
            const int mm = p + 1, M = 2 * mm;
            const std::vector<double> W = hdg::lf_prolongation_weights(m, L.topo, p);
            const double c[2] = {0.3, -1.1};
            std::vector<double> u(ne);
            for (int e = 0; e < ne; ++e) {   // flux along the owner's outward normal
                const int K = L.topo.facet_cell[2 * e], i = L.topo.facet_loc[2 * e];
                const double *x = &corners[9 * (size_t)K];
                const double tx = x[3 * ((i + 2) % 3)] - x[3 * ((i + 1) % 3)];
                const double ty = x[3 * ((i + 2) % 3) + 1] - x[3 * ((i + 1) % 3) + 1];
                u[e] = c[0] * ty - c[1] * tx;
            }
            for (int e = 0; e < ne; ++e)
                for (int d = 0; d < 2; ++d)
                    for (int k = 0; k < mm; ++k) {
                        double s = 0.0;
                        for (int j = 0; j < 5; ++j) {
                            const int f = j == 0 ? e : L.nbr[(size_t)(j - 1) * ne + e];
                            s += W[((size_t)j * M + d * mm + k) * ne + e] * u[f];
                        }
                        require(std::fabs(s - c[d]) < 1e-12, tag + " RT0: LF prolongation keeps constants");
                    }
        }
    }
    // nested RT0 spaces on flat cells: P^T S_fine P = S_coarse, and the
    // restriction lists are the transpose of the prolongation lists
    for (size_t l = 1; l < H.size(); ++l) {
        hdg::Rt0Host &F = R[l];
        const hdg::Rt0Host &C = R[l - 1];
        hdg::rt0_transfer(H[l].mesh(), F, H[l - 1].mesh(), C, H[l].par.data());
        const int nf = F.ne, nc = C.ne;
        std::vector<double> P((size_t)nf * nc, 0.0);
        for (int e = 0; e < nf; ++e)
            for (int j = 0; j < 3; ++j) P[(size_t)e * nc + F.pc[(size_t)j * nf + e]] += F.pw[(size_t)j * nf + e];
        const std::vector<double> PtSP =
            matmul(transpose(P, nf, nc), matmul(hdg::rt0_dense(F), P, nf, nf, nc), nc, nf, nc);
        const std::vector<double> Cd = hdg::rt0_dense(C);
        double d = 0.0;
        for (size_t i = 0; i < Cd.size(); ++i) d = std::fmax(d, std::fabs(PtSP[i] - Cd[i]));
        require(d < 1e-10 * max_abs(Cd), tag + " RT0: P^T S_fine P = S_coarse");
        std::vector<double> Pt((size_t)nc * nf, 0.0);
        require((int)F.crow.size() == nc + 1, tag + " RT0: restriction row count");
        for (int c = 0; c < nc; ++c)
            for (int k = F.crow[c]; k < F.crow[c + 1]; ++k) Pt[(size_t)c * nf + F.ccol[k]] += F.cw[k];
        const std::vector<double> PT = transpose(P, nf, nc);
        double t = 0.0;
        for (size_t i = 0; i < Pt.size(); ++i) t = std::fmax(t, std::fabs(Pt[i] - PT[i]));
        require(t < 1e-14, tag + " RT0: restriction is the transpose");
    }
    ok(tag + " RT0 levels");
}

template <typename F>
void expect_error(const std::string &what, F &&f) {
    try {
        f();
    } catch (const hdg::Error &e) {
        require(e.code == HDG_EINVAL && !e.msg.empty(), what + ": error code");
        ok(what + " rejected");
        return;
    }
    fail(what + ": accepted");
}

void check_errors() {
    const double xyz[12] = {0, 0, 0, 1, 0, 0, 0, 1, 0, 1, 1, 0};
    const int32_t one[3] = {0, 1, 2};
    expect_error("open mesh", [&] { hdg::build_topology(hdg_mesh{HDG_TORUS, 3, 1, 1.0, xyz, one, nullptr}); });
    const int32_t bad[3] = {0, 1, 7};
    expect_error("vertex id out of range", [&] { hdg::build_topology(hdg_mesh{HDG_TORUS, 3, 1, 1.0, xyz, bad, nullptr}); });
    const int32_t fan[9] = {0, 1, 2, 1, 0, 3, 0, 1, 3};   // edge 0-1 in three cells
    expect_error("facet in three cells", [&] { hdg::build_topology(hdg_mesh{HDG_TORUS, 4, 3, 1.0, xyz, fan, nullptr}); });
    const double sph[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    const int32_t tri[3] = {0, 1, 2};
    expect_error("RT0 on the sphere", [&] { hdg::build_rt0_level(hdg_mesh{HDG_SPHERE, 3, 1, 1.0, sph, tri, nullptr}, 1.0, true); });
}

}  // namespace

int main(int argc, char **argv) {
    try {
        check_ref_tables();
        check_errors();
        for (int a = 1; a < argc; ++a) {
            const std::vector<Level> H = read_hierarchy(argv[a]);
            const std::string tag = std::string(argv[a]).substr(std::string(argv[a]).find_last_of('/') + 1);
            for (size_t l = 0; l < H.size(); ++l) check_topology(tag + " level " + std::to_string(l), H[l]);
            const hdg_mesh fine = H.back().mesh();
            const bool unique = hdg::cells_unique_by_vertices(fine);
            require(unique == (H.back().nk > 2), tag + ": cells told apart by their vertices except on the 1 x 1 torus");
            check_p1(tag, H, 0.7);
            if (H[0].geom == HDG_TORUS) check_rt0(tag, H, 0.7);
        }
    } catch (const hdg::Error &e) {
        fail("unexpected error: " + e.msg);
    }
    std::printf("ALL OK\n");
    return 0;
}
