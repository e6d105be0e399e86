// Device kernels of the flux basis library and their launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace sdmm {

// Per Darcy subdomain (device-resident table entry).
struct DarcyDev {
    int nx, ny, N, swap, b, R, nterm, n_medge;
    // the factored system: the N cells (trapezoidal mass, half bandwidth b)
    // or, with the exact mass, Ns face pressures of half bandwidth bs
    int exact, Ns, bs, pad;
    double hx, hy, nu, mean_logk;
    int64_t off_be;     // boundary-edge arrays (2 (nx + ny) entries)
    int64_t off_cellbe; // 2 entries per cell (row-major): boundary edge ids or -1
    int64_t off_Pi;     // n_medge x R
    int64_t off_phi;    // nterm x N
    int64_t off_dofs;   // into the concatenated local->global mortar list
    int64_t off_supp;   // CSR pointer base (R + 1 entries) into supp arrays
    int64_t off_me;     // internal cell index of every mortar edge (n_medge)
};

// One basis-build unit: Darcy subdomain d, local realization k.
struct UnitDev {
    int d, k, sub, pad;
    int64_t off_xi;     // region-local collocation point (nterm values)
    int64_t off_S;      // S (R x R, column-major) in the basis cache
    int64_t off_X;      // fine responses X (N x R, internal cell order)
    int64_t off_L;      // band factor scratch (N x (b + 1))
    int64_t off_T;      // K / transmissibility scratch (4 N + n_medge)
    int64_t off_I;      // inverses of the 16 x 16 diagonal blocks of L (Np x 16)
};

struct DarcyTables {
    const DarcyDev* dar;
    const UnitDev* units;
    const int* be_cell;
    const int* be_kind;
    const double* be_len;
    const double* be_hperp;
    const int* be_medge;
    const int* be_sgn;
    const int* cell_be;
    const double* Pi;
    const double* phi;
    const double* xi;
    const int* supp_ptr;
    const int* supp_e;
    const double* supp_v;
    const int* me_cell;
    const int* order;   // unit ids grouped by shape class
    int unit_base;      // first entry of `order` this launch covers
};

// KL expansion on the device: per region the half-lengths, correlation
// lengths, amplitude, centre, kept terms and 1-D modes computed (nterm + 1
// per direction); per Darcy subdomain its cell grid and phi offset.
struct KLRegionDev {
    double ax, ay, etax, etay, sigma2, xc, yc;
    int nterm, nm;
};
struct KLSubDev {
    double x0, y0, hx, hy;
    int nx, ny, region, pad;
    int64_t off_phi;
};
// 1-D roots (w, nrm, lam1: nreg x 2 x nm_max), kept modes (ma, mb, lam2:
// nreg x nt_max) and phi of every Darcy subdomain (nterm x cells at off_phi)
hipError_t launch_kl(const KLRegionDev* reg, int nreg, const KLSubDev* sub, int nsub, int nm_max, int nt_max,
                     int max_cells, double* w, double* nrm, double* lam1, int* ma, int* mb, double* lam2, double* phi,
                     hipStream_t stream);

// Launchers (all enqueue on `stream`).

constexpr int kMaxDarcyBand = 112;   // largest padded half-bandwidth of a Darcy unit
size_t darcy_factor_lds(int bp, size_t elem);
size_t darcy_solve_lds(int bp, int R, size_t elem);
// max_np: largest padded cell count of the launch's units
// rs: right-hand sides per solve workgroup (16, 32 or 64; 0 picks the
// smallest of them that holds max_R, at most 64)
// exact != 0: the hybridized system of the exactly integrated RT0 mass (FP64)
hipError_t launch_darcy_basis_blocked(const DarcyTables& t, int n_units, int max_b, int max_R, int max_np, int rs,
                                      double* S_cache, double* X, double* Lscr, double* Iscr, double* Tscr, int exact,
                                      hipStream_t stream);
// Method S1: the band factors of the units only (mortar loads E, factor L,
// block inverses I, transmissibilities T), for per-iteration local solves
hipError_t launch_darcy_factor_only(const DarcyTables& t, int n_units, int max_b, int max_np, double* E, double* L,
                                    double* I, double* T, hipStream_t stream);
// Method S1: Y = the Darcy part of S_H x for nvec vectors x (rows of M values)
// through one local solve per (vector, Darcy subdomain); unit_of_dq[di nq + q]
// is the unit of subdomain di for realization q = slot_q[s] (slot_q may be
// null: q = s); the solutions z stay in zbuf (nvec x ndarcy x max_np); Y
// may be null (solves only)
hipError_t launch_darcy_s1_apply(const DarcyTables& t, const int* unit_of_dq, int nq, int nvec, const int* slot_q,
                                 const int32_t* active, const double* x, int M, const int64_t* sub_dof_ptr,
                                 const int64_t* sub_dofs, const double* L, const double* I, const double* T,
                                 const double* E, double* zbuf, int ndarcy, int max_np, int max_b, double* Y,
                                 int64_t SR, hipStream_t stream);
// Method S1 moments: the fine Darcy fields of the nq realizations from zbuf
// (after launch_darcy_s1_apply with x = lambda) into F (nq x (f1 + f2)), and
// their weighted sums added to sum (E[p], E[p^2], E[u], E[u^2])
hipError_t launch_darcy_s1_moments(const DarcyTables& t, const int* unit_of_dq, int nq, const double* lam, int M,
                                   const int64_t* sub_dof_ptr, const int64_t* sub_dofs, const double* zbuf,
                                   int ndarcy, int max_np, const int64_t* cell_out_off, const int64_t* edge_out_off,
                                   int64_t f1, int64_t f2, double* F, const double* weights, const int64_t* gidx,
                                   const double* colloc_w, double* sum, hipStream_t stream);
constexpr int kS1MaxR = 256;       // Method S1: mortar DOFs of one Darcy subdomain
constexpr int kS1MaxMedge = 512;   // Method S1: mortar edges of one Darcy subdomain
hipError_t launch_darcy_basis_blocked_mixed(const DarcyTables& t, int n_units, int max_b, int max_R, int max_np, int rs,
                                            double* S_cache, double* X, double* E, float* L32, float* I32,
                                            double* Tscr, float* W32, int max_refine, double refine_tol,
                                            double* max_res, int* steps, hipStream_t stream);

// Stokes: tiled band LDL^T (tile 64) of several subdomains at once.
struct StokesDev {
    int nband, nblk, w, ncol;   // ncol = R + 1
    int nvel, npre, R, nker;
    int64_t off_tiles;  // tiled band storage
    int64_t off_rhs;    // nblk*64 x ncol column-major
    int64_t off_U;      // nvel x ncol (raw velocity responses)
    int64_t off_P;      // npre x ncol
    int64_t off_map;    // band -> raw map (nband entries; pressure encoded as -1 - q)
    int64_t off_Z;      // nker x nvel
    int64_t off_q;      // CSR pointer base of the trace rows (R + 1)
    int64_t off_S;      // basis cache offset
    int64_t off_dofs;   // local->global mortar DOFs
    int64_t off_G;      // first column of this subdomain's kernel traces in G
    int64_t off_cptr;   // CSR row pointer base of the full band matrix (nband + 1)
    int64_t off_linv;   // L(J, J)^{-1} of every block column (nblk x 64 x 64)
};

// Exact RT0 mass, units too wide for the LDS window: per chunk of nu units
// (units: their ids; sdx: one StokesDev per unit, tile, right-hand-side and
// inverse offsets into the chunk's buffers), the band into zeroed tiles and
// the mortar loads into zeroed column-major right-hand sides; after the tiled
// band LDL^T solve, the solutions into X and the flux bases into S.
hipError_t launch_exact_tiles_assemble(const DarcyTables& t, const int* units, const StokesDev* sdx, int nu, int max_ld,
                                       double* tiles, double* rhs, double* Tscr, hipStream_t stream);
hipError_t launch_exact_tiles_finish(const DarcyTables& t, const int* units, const StokesDev* sdx, int nu, int max_np,
                                     int max_R, const double* rhs, double* X, double* S_cache, const double* Tscr,
                                     hipStream_t stream);
hipError_t launch_stokes_scatter(const StokesDev* sd, int ns, const int* tr_sub, const int* tr_r, const int* tr_c,
                                 const double* tr_v, int64_t ntrip, double* tiles, hipStream_t stream);
hipError_t launch_stokes_pad_identity(const StokesDev* sd, int ns, int max_nblk, double* tiles, hipStream_t stream);
// one block column J of the band LDL^T: diag (the last update of tile
// (J, J), its LDL^T and L(J, J)^{-1}), panel (the last update of the tiles
// below it, then L(I, J)) and rest (the updates of block column J to the
// tiles of columns J + 2 ..); rest of column J must finish before the diag
// launch of column J + 2
hipError_t launch_stokes_ldl_diag(const StokesDev* sd, int ns, int J, double* tiles, double* linv,
                                  hipStream_t stream);
hipError_t launch_stokes_ldl_panel(const StokesDev* sd, int ns, int J, int max_w, double* tiles, const double* linv,
                                   hipStream_t stream);
hipError_t launch_stokes_ldl_rest(const StokesDev* sd, int ns, int J, int max_w, double* tiles, hipStream_t stream);
// after the factor: the sweep tiles M (in place of L) and N (into tilesN)
hipError_t launch_stokes_sweep_tiles(const StokesDev* sd, int ns, int max_nblk, int max_w, double* tiles,
                                     double* tilesN, const double* linv, hipStream_t stream);
// x := A^{-1} x for all R + 1 columns (tmp: work array of the size of x)
hipError_t launch_stokes_solve(const StokesDev* sd, int ns, int max_nblk, int max_w, int max_ncol, const double* tiles,
                               const double* tilesN, const double* linv, double* x, double* tmp, hipStream_t stream);
// the forward step of block column J while the factor runs (any time after
// the panel launch of J, after the forward step of J - 1): reads L(I, J) and
// L(J, J)^{-1}, updates x in place and writes L^{-1}-scaled block J to tmp,
// bit for bit what the forward sweep of launch_stokes_solve does after the
// factor; launch_stokes_solve_back then finishes the solve.
hipError_t launch_stokes_fwd_early(const StokesDev* sd, int ns, int J, int max_w, int max_ncol, const double* tiles,
                                   const double* linv, double* x, double* tmp, hipStream_t stream);
// the backward sweep tiles N(J, .) of block row J (the sweep-tile kernel's
// bits), once the panel launch of J - 1 and the diag launch of J are done
hipError_t launch_stokes_sweep_row(const StokesDev* sd, int ns, int J, int max_w, const double* tiles, double* tilesN,
                                   const double* linv, hipStream_t stream);
hipError_t launch_stokes_solve_back(const StokesDev* sd, int ns, int max_nblk, int max_w, int max_ncol,
                                    const double* tiles, const double* tilesN, const double* linv, double* x,
                                    double* tmp, hipStream_t stream);
// FP64 iterative refinement of the band solves: res = b - A x with the
// assembled band matrix (tiles0; fixed summation order), then x += d after
// d = A^{-1} res.
hipError_t launch_stokes_residual(const StokesDev* sd, int ns, int max_nblk, int max_ncol, const double* tiles0,
                                  const double* b, const double* x, double* res, hipStream_t stream);
hipError_t launch_add_inplace(double* x, const double* d, int64_t n, hipStream_t stream);
// x[0 .. n) = 0 with a kernel (graph-safe, unlike a memset node)
hipError_t launch_fill_zero(double* x, int64_t n, hipStream_t stream);
hipError_t launch_stokes_finish(const StokesDev* sd, int ns, int max_ncol, int max_R, const double* rhs, const int* bmap,
                                const double* uD, const int64_t* uD_off, const double* Z, const int* q_ptr,
                                const int* q_col, const double* q_val, const int64_t* dofs, double* U, double* P,
                                double* S_cache, double* g, double* G, int M, hipStream_t stream);

// Interface CG
struct CgArgs {
    int64_t n;            // realizations in the batch
    int M, nsub, nregion, nker;
    const int64_t* gidx;
    const int32_t* g2l;   // n_real x n_region
    const int* sub_R;
    const int64_t* sub_dof_ptr;
    const int64_t* sub_dofs;
    const int* sub_region;   // -1 for Stokes
    const int64_t* sub_Sbase;
    const double* S_cache;
    const double* g;
    const double* G;         // M x nker (column-major)
    const double* GtGinv;    // nker x nker
    double* lam;
    double* r;
    double* p;
    double* rr;
    double* r0;
    double* pend;         // per slot: lambda update held back one iteration (cg_update2)
    int32_t* iters;
    double* relres;
    int32_t* status;
    int32_t* active;
    int32_t* any_active;
    const int* Grow;         // rows of G with non-zero entries (floating subdomains)
    const double* Gval;      // nGrow x nker values of those rows
    int nGrow;
    double rtol;
    int max_iter;
    // slots: the CG state arrays (r, p, rr, r0, iters, relres, status, active)
    // have one row per slot; slot l holds batch realization slot_q[l], whose
    // lambda row and outputs are at that batch position
    const int* slot_q;
    const int* init_slots;   // slots cg_init starts
    int32_t* iters_out;      // batch outputs, written when a realization stops (may be null)
    double* relres_out;
    int32_t* status_out;
};

hipError_t launch_validate_index(const int64_t* gidx, int64_t n, int64_t nreal, int32_t* bad, hipStream_t stream);
// starts the CG of the `count` slots listed in a.init_slots
hipError_t launch_cg_init(const CgArgs& a, int64_t count, hipStream_t stream);
hipError_t launch_cg_apply_mfma(const CgArgs& a, const double* x, double* Y, int64_t SR, const int4* work, int nwork,
                                const int* perm, int max_R, hipStream_t stream, hipEvent_t t0 = nullptr,
                                hipEvent_t t1 = nullptr);
hipError_t launch_gather_global(const double* Y, int64_t SR, const int* pos, int M, int64_t n, double* y,
                                hipStream_t stream);
// t0/t1, when given, receive the start and end time stamps of the kernel's own
// dispatch (hipExtLaunchKernel), so their interval excludes launch gaps.
hipError_t launch_cg_update2(const CgArgs& a, const double* Y, int64_t SR, const int* pos, hipStream_t stream,
                             hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr);
hipError_t launch_count_active(const int32_t* active, int64_t n, int32_t* count, hipStream_t stream);
// copy finished realizations (CG slot slot[q]) to their callers' buffers
hipError_t launch_stream_gather(const double* lam, int M, const int* slot, double* const* dst_lam, const int32_t* it,
                                const double* rel, const int32_t* stat, int32_t* const* dst_it,
                                double* const* dst_rel, int32_t* const* dst_st, int n, hipStream_t stream);

// Moments
struct MomArgs {
    int64_t n;
    int M, nsub, nregion, nker;
    const int64_t* gidx;
    const int32_t* g2l;
    const double* weights;   // n (or null: use colloc weights)
    const double* colloc_w;
    const double* lam;       // n x M
    const int* sub_R;
    const int64_t* sub_dof_ptr;
    const int64_t* sub_dofs;
    const int* sub_region;
    const int* sub_ker;      // kernel columns of each subdomain (0 if not floating)
    const int* sub_Gcol;     // first column in alpha of each subdomain
    const int64_t* sub_Abase;   // accumulator base of each subdomain (a and M for every local k)
    const int* sub_nlocal;
    const double* alpha;     // n x nker
    double* acc;             // accumulators
    double* lam1;
    double* lam2;
    double* wsum;
};
hipError_t launch_alpha(const CgArgs& a, const double* Slam, double* alpha, hipStream_t stream);
hipError_t launch_accumulate_chunks(const MomArgs& m, const int4* awork, int nawork, const int* perm,
                                    const int64_t* slot, double* part, const int* pair_sub, const int* pair_k,
                                    const int* pair_item0, int npairs, int max_ext, hipStream_t stream);
hipError_t launch_darcy_moments_impl(const DarcyTables& t, const int* unit_of_dk, const int* d_nlocal, int n_darcy,
                                     int max_nout, int max_units_per_d, const int64_t* d_Abase, const double* acc,
                                     const double* X, int max_R, const int64_t* cell_out_off,
                                     const int64_t* edge_out_off, double* p1, double* p2, double* u1, double* u2,
                                     hipStream_t stream);
hipError_t launch_stokes_moments_impl(const StokesDev* sd, int ns, int max_nout, const int64_t* s_Abase,
                                      const double* acc, const double* wsum, const double* U, const double* P,
                                      const double* Z, const int64_t* u_out_off, const int64_t* p_out_off, int max_ext,
                                      double* u1, double* u2, double* p1, double* p2, hipStream_t stream);

// Workspace of the allocation-free CG entry point: kNoAllocScratchBytes of
// device memory per GPU, a fixed array in the code object.
// noalloc_scratch_setup(device) resolves that GPU's copy (device must be
// current; once per device, later calls return at once);
// noalloc_scratch_ptr(device) gives its address, or null before set-up.
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
hipError_t noalloc_scratch_setup(int device);
void* noalloc_scratch_ptr(int device);

}  // namespace sdmm
