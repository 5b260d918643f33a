// Host-side declarations of the HDG trace-multigrid library: errors, mesh
// topology, reference-element tables and the P1 / RT0 coarse-level builders.
// Plain C++ (no HIP), so the builders also compile with a host compiler
// alone, for instance under the address and undefined-behaviour sanitizers.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/hdg.h"

namespace hdg {

// ------------------------------------------------------------------ errors
void set_error(const std::string &msg);

struct Error {
    int code;
    std::string msg;
};

#define HDG_REQUIRE(cond, msg)                                                       \
    do {                                                                             \
        if (!(cond)) throw ::hdg::Error{HDG_EINVAL, (msg)};                          \
    } while (0)

// ------------------------------------------------------------------ host topology
struct Topology {
    int n_cell = 0, n_facet = 0;
    std::vector<int32_t> cell_facet;  // [n_cell][3]
    std::vector<int8_t> cell_rev;     // [n_cell][3] 1 when the cell runs against the facet direction
    std::vector<int32_t> facet_cell;  // [n_facet][2] owner, other
    std::vector<int32_t> facet_loc;   // [n_facet][2]
    std::vector<int32_t> facet_vert;  // [n_facet][2] start, end
};
Topology build_topology(const hdg_mesh &mesh);

// Unwrapped corner coordinates [n_cell][3][3].
std::vector<double> cell_corners(const hdg_mesh &mesh);

// ------------------------------------------------------------------ reference tables
// Lagrange basis at the equispaced lattice of the reference triangle and the
// integrals the per-cell assembly needs.  Sizes: n = (p+1)(p+2)/2, m = p+1,
// nq = (p+3)^2 collapsed Gauss points.
struct RefTables {
    int p = 0, n = 0, m = 0, nq = 0;
    std::vector<double> M;     // [n][n]      int phi_i phi_j
    std::vector<double> G;     // [2][n][n]   int phi_i d_r phi_j
    std::vector<double> E;     // [3][n][n]   int_0^1 phi_i phi_j ds on facet f
    std::vector<double> T;     // [3][n][m]   int_0^1 phi_i mu_k ds on facet f
    std::vector<double> F;     // [m][m]      int_0^1 mu_k mu_l ds
    std::vector<double> qx;    // [nq][2]     quadrature points
    std::vector<double> qw;    // [nq]        weights (sum 1/2)
    std::vector<double> Phi;   // [nq][n]     basis values at the points
};
RefTables build_ref_tables(int p);

// ------------------------------------------------------------------ P1 levels (host)
struct P1Host {
    int n = 0;
    std::vector<int32_t> rowptr, col;  // CSR of S_c without the diagonal
    std::vector<double> val;
    std::vector<double> diag;
};
P1Host assemble_p1(const hdg_mesh &mesh, double kappa);
P1Host galerkin_from_rows(int ne, int m, int nv, const std::vector<double> &rows, const std::vector<int32_t> &nbr,
                          const std::vector<int32_t> &facet_vert);
P1Host galerkin_coarsen(const P1Host &fine, const int32_t *parents, int nc);
// matrix [n][n] (row-major, n the finest level's size) of one P1 multigrid V-cycle over the
// levels ops (coarse to fine) with damped Jacobi (nu sweeps, damping omega) and the parent-pair
// transfers: the linear map the V-cycle applies to the finest level's right-hand side
std::vector<double> p1_vcycle_matrix(const std::vector<P1Host> &ops, const int32_t *const *parents, int nu,
                                     double omega);
// in-place inverse of a dense SPD matrix [n][n]; returns false when not positive definite
bool spd_inverse(std::vector<double> &a, int n);
// in-place inverse of a dense matrix [n][n] (Gauss-Jordan, partial pivoting); false when singular
bool invert_dense(std::vector<double> &a, int n);

// ------------------------------------------------------------------ RT0 levels (host), Lax-Friedrichs flux
constexpr int RT_PV = 8;   // most facets around one vertex (vertex-patch size)

struct Rt0Host {
    int ne = 0, nv = 0;
    Topology topo;
    std::vector<int32_t> nbr;     // [4][ne] other facets of the owner, then of the second cell
    std::vector<double> val;      // [5][ne] S_c row of each facet: diagonal, then the nbr slots
    std::vector<int32_t> pf;      // [RT_PV][nv] facets touching each vertex, -1 padded
    std::vector<double> pinv;     // [RT_PV * RT_PV][nv] inverse of the patch block (zero padded)
    std::vector<int32_t> fs;      // [2][ne] patch slot v * RT_PV + j of the facet's two ends
    std::vector<int32_t> pc;      // [3][ne] coarse facets of the next coarser level feeding this facet
    std::vector<double> pw;       // [3][ne] their weights (exact flux transfer)
    std::vector<int32_t> crow, ccol;   // transpose of (pc, pw) over the coarser level's facets
    std::vector<double> cw;
};
// S_c = (1/kappa)(M_RT + kappa^2 D_RT) on the torus mesh, patches and their inverses
Rt0Host build_rt0_level(const hdg_mesh &mesh, double kappa, bool patches);
// true when every cell of the mesh is determined by its three vertex ids
bool cells_unique_by_vertices(const hdg_mesh &mesh);
// inclusion RT0(coarse) -> RT0(fine) of a uniform refinement (fills fine.pc / pw / crow / ccol / cw)
void rt0_transfer(const hdg_mesh &fine_mesh, Rt0Host &fine, const hdg_mesh &coarse_mesh, const Rt0Host &coarse,
                  const int32_t *parents);
// dense S_c of a level [ne][ne]
std::vector<double> rt0_dense(const Rt0Host &L);
// pi: RT0 fluxes -> LF trace nodes, weights [5][2m][ne] over the facet-row patch (facet, then nbr slots)
std::vector<double> lf_prolongation_weights(const hdg_mesh &mesh, const Topology &topo, int p);

}  // namespace hdg
