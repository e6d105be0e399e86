// Host-side problem setup: layout, mortar maps, KL modes, collocation,
// Darcy subdomain descriptors and Stokes subdomain operators.
#pragma once
#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "../../include/sdmm.h"

namespace sdmm {

struct Sub {
    int type;  // 0 Stokes, 1 Darcy
    double x0, x1, y0, y1;
    int nx, ny;
    double hx, hy;
    int region;
};

struct Iface {
    int i, j, kind;   // kind 0 ss, 1 sd, 2 dd
    int horizontal;   // 1: y = coord, tangential coordinate x
    double coord, a, b;
    int ncomp, nelem, deg, off, nnode, ndof;
    double H;
    // integral over [t0, t1] of every scalar node shape times g (g given on
    // the 3 Gauss points of each refinement piece through a callback)
    template <class G>
    void node_integrals(double t0, double t1, const G& g, double* out) const;
};

struct KLRegion {
    std::vector<int> ma, mb;        // 1-D mode indices of the kept 2-D modes
    std::vector<double> lam;        // sigma^2 lambda_a lambda_b
    std::vector<double> wx, nx_, wy, ny_;  // 1-D roots and norms
    std::vector<int> px, py;        // parity 0 even / 1 odd
    double xc, yc;
};

struct MedgeTerm { int dof; double val; };

// One Darcy subdomain as the basis kernels see it.
struct DarcyHost {
    int sub;
    int nx, ny, N, swap, b;   // swap: internal order is y-fastest (nx > ny)
    // factored system: the N cells (half bandwidth b), or with the exact
    // RT0 mass the Ns = nyi (2 nxi + 1) + nxi face pressures (bs = 2 nxi + 1)
    int exact, Ns, bs;
    double hx, hy;
    int R;
    // boundary edges: 2(nx+ny), ordered bottom, top, left, right
    std::vector<int> be_cell;      // row-major cell index
    std::vector<int> be_kind;      // 0 mortar, 1 Dirichlet, 2 no-flow
    std::vector<double> be_len, be_hperp;
    std::vector<int> be_medge;     // index into the mortar edge list or -1
    std::vector<int> be_sgn;       // +1 if the outward normal is +x / +y
    std::vector<int> be_edge;      // RT0 edge index
    int n_medge;
    std::vector<double> Pi;        // n_medge x R edge averages of the mortar functions
    int nterm;
    double mean_logk;
};

// One Stokes subdomain: saddle operator in band order.
struct StokesHost {
    int sub;
    int nx, ny, nvel, npre;   // raw counts
    int R;
    int floating;
    int nband;                // unknowns in the band system
    int bw;                   // half bandwidth
    std::vector<int> band_kind;   // 0 velocity, 1 pressure
    std::vector<int> band_raw;    // raw velocity DOF (2 node + comp) or pressure node
    // band matrix entries (lower part, including the diagonal) as triplets
    std::vector<int> ar, ac;
    std::vector<double> av;
    // right-hand sides: R basis loads (-Q^T e_j) and one complementary load
    std::vector<double> rhs;  // nband x (R + 1), column-major
    // trace rows: Q restricted to band unknowns (CSR over R rows)
    std::vector<int> q_ptr, q_col;
    std::vector<double> q_val;
    std::vector<double> gD;   // Q_D u_D (Dirichlet part of g), R values
    std::vector<double> uD;   // raw velocity with Dirichlet values (zero elsewhere)
    std::vector<double> Z;    // nband x nker kernel basis (velocity rows), orthonormal
    int nker;
};

struct Problem {
    sdmm_problem in;
    // copies of the input arrays
    std::vector<Sub> subs;
    int n_stokes = 0, n_darcy = 0;
    std::vector<Iface> ifaces;
    int M = 0;
    std::vector<std::vector<int>> sub_ifaces;
    std::vector<int64_t> sub_ptr, sub_dofs, sub_sign;
    std::vector<std::vector<int>> sub_dof_off;  // per subdomain, per iface listed: local offset
    // regions
    int n_region = 0;
    std::vector<double> region_rect, region_sigma2, region_eta, region_mean;
    std::vector<int> region_nterm;
    std::vector<KLRegion> kl;
    // collocation
    int nterm = 0;
    std::vector<int> dim_off;
    int64_t nreal = 0;
    std::vector<double> node_x;
    std::vector<int32_t> ids;        // nreal x nterm
    std::vector<double> weights;     // nreal
    std::vector<std::vector<int32_t>> local_ids;  // per region: L_r x nterm_r
    std::vector<int32_t> g2l;        // nreal x n_region
    std::vector<int> nlocal;
    // subdomain operators
    std::vector<DarcyHost> darcy;
    std::vector<StokesHost> stokes;
    // FETI
    int n_kernel = 0;
};

// Builds everything; returns an empty string or an error message.
std::string build_problem(const sdmm_problem& p, Problem& out);

}  // namespace sdmm
