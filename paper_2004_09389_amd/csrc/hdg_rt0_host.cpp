// Host set-up of the Lax-Friedrichs coarse space: lowest-order Raviart-Thomas
// (RT0) levels on the nested torus hierarchy, their transfers, vertex patches
// and the prolongation onto the vector trace (non-nested multigrid section,
// Lax-Friedrichs case; Eq. coarse_problem_LF).
//
// RT0 unknown of facet e: the flux of the field through e along the owner
// cell's outward normal.  On cell K the basis function of local facet i
// (opposite local vertex v_i) is sigma_i (x - v_i) / (2|K|), sigma_i = +1 when
// K owns the facet and -1 otherwise: its flux through facet i is sigma_i and
// through the other two facets zero; its divergence is sigma_i / |K|.
#include <algorithm>
#include <array>
#include <cmath>
#include <map>

#include "hdg_host.h"

namespace hdg {

namespace {

struct CellGeo {
    double x[3][2];   // unwrapped corners
    double area;
};

CellGeo cell_geo(const std::vector<double> &corners, int K) {
    CellGeo g;
    for (int k = 0; k < 3; ++k)
        for (int d = 0; d < 2; ++d) g.x[k][d] = corners[(size_t)9 * K + 3 * k + d];
    g.area = 0.5 * ((g.x[1][0] - g.x[0][0]) * (g.x[2][1] - g.x[0][1]) -
                    (g.x[1][1] - g.x[0][1]) * (g.x[2][0] - g.x[0][0]));
    return g;
}

// value of basis function i of the cell at point X (same unwrapped coordinates)
void rt_basis(const CellGeo &g, int i, double sigma, const double X[2], double out[2]) {
    for (int d = 0; d < 2; ++d) out[d] = sigma * (X[d] - g.x[i][d]) / (2.0 * g.area);
}

// outward unit normal and length of local facet i (from corner i+1 to i+2, counter-clockwise)
void facet_normal(const CellGeo &g, int i, double n[2], double &len) {
    const double tx = g.x[(i + 2) % 3][0] - g.x[(i + 1) % 3][0], ty = g.x[(i + 2) % 3][1] - g.x[(i + 1) % 3][1];
    len = std::sqrt(tx * tx + ty * ty);
    n[0] = ty / len;
    n[1] = -tx / len;
}

// slot of local facet j of the cell on side s of facet e (local index i there) in e's row patch
int patch_slot(int s, int i, int j) { return j == i ? 0 : 2 * s + (j - i + 3) % 3; }

}  // namespace

bool cells_unique_by_vertices(const hdg_mesh &mesh) {
    std::map<std::array<int, 3>, int> seen;
    for (int K = 0; K < mesh.n_cell; ++K) {
        std::array<int, 3> v{mesh.cell_vert[3 * K], mesh.cell_vert[3 * K + 1], mesh.cell_vert[3 * K + 2]};
        std::sort(v.begin(), v.end());
        if (v[0] == v[1] || v[1] == v[2]) return false;
        if (!seen.emplace(v, K).second) return false;
    }
    return true;
}

Rt0Host build_rt0_level(const hdg_mesh &mesh, double kappa, bool patches) {
    HDG_REQUIRE(mesh.geom == HDG_TORUS, "the RT0 coarse space is built on the torus only");
    Rt0Host L;
    L.topo = build_topology(mesh);
    const Topology &T = L.topo;
    const int ne = T.n_facet, nk = mesh.n_cell, nv = mesh.n_vert;
    L.ne = ne;
    L.nv = nv;
    const std::vector<double> corners = cell_corners(mesh);
    L.nbr.assign((size_t)4 * ne, -1);
    L.val.assign((size_t)5 * ne, 0.0);
    for (int e = 0; e < ne; ++e)
        for (int s = 0; s < 2; ++s) {
            const int K = T.facet_cell[2 * e + s], i = T.facet_loc[2 * e + s];
            for (int jj = 1; jj < 3; ++jj) L.nbr[(size_t)(2 * s + jj - 1) * ne + e] = T.cell_facet[3 * K + (i + jj) % 3];
        }
    // cell contributions: (1/kappa) [ (phi_a, phi_b) + kappa^2 (div phi_a, div phi_b) ]; the mass
    // integrand is quadratic, integrated exactly by the edge-midpoint rule |K|/3 sum_edges g(mid)
    for (int K = 0; K < nk; ++K) {
        const CellGeo g = cell_geo(corners, K);
        double sg[3];
        for (int i = 0; i < 3; ++i) sg[i] = T.cell_rev[3 * K + i] ? -1.0 : 1.0;
        double Mk[3][3] = {};
        for (int q = 0; q < 3; ++q) {
            const double X[2] = {0.5 * (g.x[(q + 1) % 3][0] + g.x[(q + 2) % 3][0]),
                                 0.5 * (g.x[(q + 1) % 3][1] + g.x[(q + 2) % 3][1])};
            double ph[3][2];
            for (int i = 0; i < 3; ++i) rt_basis(g, i, sg[i], X, ph[i]);
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) Mk[a][b] += g.area / 3.0 * (ph[a][0] * ph[b][0] + ph[a][1] * ph[b][1]);
        }
        for (int a = 0; a < 3; ++a) {
            const int e = T.cell_facet[3 * K + a];
            const int s = T.cell_rev[3 * K + a] ? 1 : 0;
            HDG_REQUIRE(T.facet_cell[2 * e + s] == K, "inconsistent RT0 facet orientation");
            for (int b = 0; b < 3; ++b) {
                const double v = (Mk[a][b] + kappa * kappa * sg[a] * sg[b] / g.area) / kappa;
                L.val[(size_t)patch_slot(s, a, b) * ne + e] += v;
            }
        }
    }
    if (patches) {
        std::vector<std::vector<int>> inc(nv);
        for (int e = 0; e < ne; ++e) {
            inc[T.facet_vert[2 * e]].push_back(e);
            if (T.facet_vert[2 * e + 1] != T.facet_vert[2 * e]) inc[T.facet_vert[2 * e + 1]].push_back(e);
        }
        L.pf.assign((size_t)RT_PV * nv, -1);
        L.pinv.assign((size_t)RT_PV * RT_PV * nv, 0.0);
        L.fs.assign((size_t)2 * ne, -1);
        auto entry = [&](int row, int col) {   // S_c[row][col] from the row storage
            double v = row == col ? L.val[row] : 0.0;
            for (int j = 0; j < 4; ++j)
                if (L.nbr[(size_t)j * ne + row] == col) v += L.val[(size_t)(j + 1) * ne + row];
            return v;
        };
        for (int v = 0; v < nv; ++v) {
            const int np = (int)inc[v].size();
            HDG_REQUIRE(np >= 1 && np <= RT_PV, "RT0 vertex patch with more than 8 facets");
            std::vector<double> A((size_t)np * np);
            for (int a = 0; a < np; ++a) {
                L.pf[(size_t)a * nv + v] = inc[v][a];
                for (int b = 0; b < np; ++b) A[(size_t)a * np + b] = entry(inc[v][a], inc[v][b]);
                const int e = inc[v][a];
                const int end = T.facet_vert[2 * e] == v ? 0 : 1;
                L.fs[(size_t)end * ne + e] = v * RT_PV + a;
            }
            HDG_REQUIRE(invert_dense(A, np), "singular RT0 vertex-patch block");
            for (int a = 0; a < np; ++a)
                for (int b = 0; b < np; ++b) L.pinv[(size_t)(a * RT_PV + b) * nv + v] = A[(size_t)a * np + b];
        }
        for (int e = 0; e < ne; ++e)
            if (L.fs[(size_t)ne + e] < 0) L.fs[(size_t)ne + e] = L.fs[e];   // both ends at one vertex: counted once
    }
    return L;
}

std::vector<double> rt0_dense(const Rt0Host &L) {
    const int ne = L.ne;
    std::vector<double> A((size_t)ne * ne, 0.0);
    for (int e = 0; e < ne; ++e) {
        A[(size_t)e * ne + e] += L.val[e];
        for (int j = 0; j < 4; ++j) A[(size_t)e * ne + L.nbr[(size_t)j * ne + e]] += L.val[(size_t)(j + 1) * ne + e];
    }
    return A;
}

void rt0_transfer(const hdg_mesh &fine_mesh, Rt0Host &F, const hdg_mesh &coarse_mesh, const Rt0Host &C,
                  const int32_t *parents) {
    HDG_REQUIRE(parents, "parents must be given for every level above the coarsest");
    std::map<std::array<int, 3>, int> cell_of;
    for (int K = 0; K < coarse_mesh.n_cell; ++K) {
        std::array<int, 3> v{coarse_mesh.cell_vert[3 * K], coarse_mesh.cell_vert[3 * K + 1],
                             coarse_mesh.cell_vert[3 * K + 2]};
        std::sort(v.begin(), v.end());
        cell_of[v] = K;
    }
    const std::vector<double> fc = cell_corners(fine_mesh), cc = cell_corners(coarse_mesh);
    const double period = coarse_mesh.period;
    const int ne = F.ne;
    F.pc.assign((size_t)3 * ne, 0);
    F.pw.assign((size_t)3 * ne, 0.0);
    std::vector<std::vector<std::pair<int, double>>> ch(C.ne);
    for (int e = 0; e < ne; ++e) {
        const int Kf = F.topo.facet_cell[2 * e], i = F.topo.facet_loc[2 * e];
        std::array<int, 3> cv{-1, -1, -1};
        int ncv = 0;
        for (int k = 0; k < 3; ++k)
            for (int h = 0; h < 2; ++h) {
                const int v = parents[2 * fine_mesh.cell_vert[3 * Kf + k] + h];
                bool have = false;
                for (int q = 0; q < ncv; ++q) have |= cv[q] == v;
                if (!have) {
                    HDG_REQUIRE(ncv < 3, "fine cell does not lie in one coarse cell");
                    cv[ncv++] = v;
                }
            }
        HDG_REQUIRE(ncv == 3, "fine cell does not lie in one coarse cell");
        std::sort(cv.begin(), cv.end());
        auto it = cell_of.find(cv);
        HDG_REQUIRE(it != cell_of.end(), "parent cell of a fine cell not found");
        const int Kc = it->second;
        const CellGeo gf = cell_geo(fc, Kf), gc = cell_geo(cc, Kc);
        double nrm[2], len;
        facet_normal(gf, i, nrm, len);
        double mid[2], cen[2];
        for (int d = 0; d < 2; ++d) {
            mid[d] = 0.5 * (gf.x[(i + 1) % 3][d] + gf.x[(i + 2) % 3][d]);
            cen[d] = (gc.x[0][d] + gc.x[1][d] + gc.x[2][d]) / 3.0;
            mid[d] -= period * std::round((mid[d] - cen[d]) / period);   // coarse cell's periodic image
        }
        for (int j = 0; j < 3; ++j) {
            const double sg = C.topo.cell_rev[3 * Kc + j] ? -1.0 : 1.0;
            double ph[2];
            rt_basis(gc, j, sg, mid, ph);
            const double w = len * (ph[0] * nrm[0] + ph[1] * nrm[1]);
            const int cf = C.topo.cell_facet[3 * Kc + j];
            F.pc[(size_t)j * ne + e] = cf;
            F.pw[(size_t)j * ne + e] = w;
            ch[cf].push_back({e, w});
        }
    }
    F.crow.assign(C.ne + 1, 0);
    F.ccol.clear();
    F.cw.clear();
    for (int c = 0; c < C.ne; ++c) {
        for (auto &pr : ch[c]) {
            F.ccol.push_back(pr.first);
            F.cw.push_back(pr.second);
        }
        F.crow[c + 1] = (int)F.ccol.size();
    }
}

std::vector<double> lf_prolongation_weights(const hdg_mesh &mesh, const Topology &T, int p) {
    const int m = p + 1, M = 2 * m, ne = T.n_facet;
    const std::vector<double> corners = cell_corners(mesh);
    std::vector<double> pw((size_t)5 * M * ne, 0.0);
    for (int e = 0; e < ne; ++e)
        for (int s = 0; s < 2; ++s) {
            const int K = T.facet_cell[2 * e + s], i = T.facet_loc[2 * e + s];
            const CellGeo g = cell_geo(corners, K);
            for (int k = 0; k < m; ++k) {
                // global node k at parameter k/p along the facet; the second cell runs it backwards
                const double t = s == 0 ? (double)k / p : 1.0 - (double)k / p;
                double X[2];
                for (int d = 0; d < 2; ++d)
                    X[d] = g.x[(i + 1) % 3][d] + t * (g.x[(i + 2) % 3][d] - g.x[(i + 1) % 3][d]);
                for (int j = 0; j < 3; ++j) {
                    const double sg = T.cell_rev[3 * K + j] ? -1.0 : 1.0;
                    double ph[2];
                    rt_basis(g, j, sg, X, ph);
                    const int slot = patch_slot(s, i, j);
                    for (int d = 0; d < 2; ++d) pw[((size_t)slot * M + d * m + k) * ne + e] += 0.5 * ph[d];
                }
            }
        }
    return pw;
}

}  // namespace hdg
