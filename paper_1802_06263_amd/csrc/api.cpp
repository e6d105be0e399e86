// C ABI of the flux basis library: host orchestration of the HIP kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/sdmm.h"
#include "kernels.hpp"
#include "problem.hpp"

using namespace sdmm;

namespace {

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    const sdmm_alloc* al = nullptr;   // the allocator that gave p (null: hipMalloc)
    int dev = 0;
    ~DevBuf() { release(); }
    void release() {
        if (p) {
            if (al)
                al->release(p, bytes, dev, al->user);
            else
                (void)hipFree(p);
        }
        p = nullptr;
        bytes = 0;
        al = nullptr;
    }
    template <class T>
    T* as() const { return reinterpret_cast<T*>(p); }
};

}  // namespace

// Realization groups of the grouped operator: the batch positions sorted by
// local index per region (perm), the operator work items (work) and the
// moment work items (awork, with their scratch offsets and first item per
// (subdomain, local realization) pair).
struct Groups {
    DevBuf d_work, d_perm, d_awork, d_slot, d_item0;
    std::vector<int4> h_work, h_awork;
    std::vector<int> h_perm, h_item0;
    std::vector<int64_t> h_slot;
    int nwork = 0, nawork = 0;
    int64_t part_total = 0;
};

constexpr int kMaxLanes = 2;   // CG lanes: halves of the slots on their own streams
constexpr int kXcds = 8;        // XCDs of an MI355X; a launch deals its workgroups to them in turn

// A CG stream (continuous batching): a fixed number of CG slots that
// realizations of any number of submitted requests occupy as they free up.
// Slot l keeps its lambda, iteration count, residual and status at row l of
// the stream's own arrays; finished realizations are copied to their
// request's buffers when they leave their slot.
struct CgStream {
    int64_t S = 0;
    double rtol = 1e-8;
    int32_t max_iter = 1;
    hipStream_t st = nullptr;
    DevBuf r, p, Y, rr, r0, pend, relres, iters, status, active, any, slot_q, init, lam;
    DevBuf g_slot, g_lam, g_it, g_rel, g_st;   // gather lists of finished realizations
    Groups G;
    std::vector<int> init_h, sel;
    std::vector<int64_t> slot_g, slot_ticket;
    std::vector<int> slot_row;
    std::vector<int32_t> act;
    struct Pending {
        int64_t ticket, gidx;
        int row;
    };
    std::deque<Pending> queue;
    struct Req {
        double* lam;
        int32_t* it;
        double* rel;
        int32_t* st;
        int64_t remaining;
    };
    std::map<int64_t, Req> reqs;
    int64_t next_ticket = 1, in_work = 0, occupied = 0, groups_run = 0;
};


// Which flux bases the interface operator and the moments use: by default
// the stochastic basis (Method S3: every local realization of the
// collocation grid, pairs (i, k) and the global->local table); a
// deterministic basis built for a batch (Method S2) gives each realization
// of the batch its own local index in every region.
struct BasisView {
    std::vector<int> pair_sub, pair_k;   // (subdomain, local index) pairs
    std::vector<int32_t> g2l;            // rows by batch position, n_region columns
    std::vector<int> nlocal;             // local indices per region
    DevBuf d_pair_sub, d_pair_k, d_sub_Sbase, d_sub_Abase;
    double* S = nullptr;                 // the basis blocks
};

// Method S2 state: the batch of the last deterministic solve and its bases.
// A chunk of exact-mass units too wide for the LDS window, built together
// through the tiled band LDL^T (entries first .. first + count - 1 of the
// unit and StokesDev lists; the chunk's doubles of tiles, right-hand sides
// and inverses).
struct WideChunk {
    int first, count, max_nblk, max_w, max_ncol, max_ld, max_np;
    int64_t tiles, rhs, linv;
};

struct DetBatch {
    int64_t n = 0, cap = 0;
    std::vector<WideChunk> wide_chunks;   // the batch's wide units (exact mass)
    DevBuf d_wide_sdx, d_wide_units;
    std::vector<double> y;               // n x n_term points of the batch
    std::vector<UnitDev> units;
    std::vector<int> chunk_start;        // unit ranges built per launch (scratch reused)
    DevBuf d_units, d_order, d_xi, d_pos, d_S, d_X, d_E, d_W32, d_L, d_L32, d_I, d_I32, d_T, d_refine;
    DevBuf d_unit_of_dk, d_dnlocal, d_dAbase, d_sum, d_tmp;
    DevBuf d_z, d_F, d_s1work, d_s1perm;   // Method S1: local solutions, fields, Stokes work list
    int s1_nwork = 0;
    int64_t S_total = 0, X_total = 0, L_chunk = 0, T_chunk = 0, I_chunk = 0, A_base = 0;
    int precision = SDMM_PREC_FP64;
    bool valid = false;
    BasisView view;
};

// State of one problem of a context (every call names its problem id).
struct Prob {
    int device = 0;
    const sdmm_alloc* alloc = nullptr;   // the context's allocator, or null
    int method = SDMM_METHOD_STOCHASTIC;
    bool host_only = false;  // device -1: problem setup and maps only
    std::string err;
    bool have_problem = false;
    bool basis_built = false;
    bool stokes_built = false;
    int built_precision = -1;
    Problem P;
    // sizes
    int max_b = 0, max_R = 0, max_Rd = 0, max_ext = 0;
    int64_t n_units = 0;
    std::vector<UnitDev> units;
    // Darcy units grouped by shape class (padded band bp, padded R): each
    // class is one launch with LDS sized for it, on its own stream
    struct UnitClass {
        int base, count, bp, Rs, np;   // np: largest padded row count of the class
        int rs[2];                     // solve group width per precision (FP64, mixed); 0: smallest holding Rs
    };
    std::vector<UnitClass> classes;
    std::vector<int> h_order;
    DevBuf d_order;
    std::vector<hipStream_t> class_streams;
    std::vector<hipEvent_t> class_events;
    std::vector<int64_t> sub_Sbase, sub_Abase;
    std::vector<int> sub_R, sub_region, sub_ker, sub_Gcol, sub_nlocal;
    std::vector<StokesDev> sdev;
    int max_nblk = 0, max_w = 0, max_ncol = 0, max_nout_d = 0, max_nout_s = 0, max_units_per_d = 0;
    int64_t n_trip = 0;
    int64_t S_total = 0, X_total = 0, L_total = 0, T_total = 0, A_total = 0, I_total = 0;
    int64_t field_size[5] = {0, 0, 0, 0, 0};
    std::vector<int64_t> cell_out_off, edge_out_off, u_out_off, p_out_off;
    std::vector<int> pair_sub, pair_k;
    // device buffers
    DevBuf d_dar, d_units, d_be_cell, d_be_kind, d_be_len, d_be_hperp, d_be_medge, d_be_sgn, d_cell_be, d_Pi, d_phi,
        d_xi, d_supp_ptr, d_supp_e, d_supp_v, d_me_cell;
    DevBuf d_S, d_X, d_L, d_T, d_L32, d_W32, d_E, d_refine, d_I, d_I32;
    DevBuf d_sdev, d_tiles, d_rhs, d_U, d_P, d_bmap, d_Z, d_q_ptr, d_q_col, d_q_val, d_uD, d_uD_off, d_tr_sub, d_tr_r,
        d_tr_c, d_tr_v, d_rhs0, d_res, d_tiles0, d_tilesN, d_linv, d_stmp;
    DevBuf d_g, d_G, d_GtGinv, d_Grow, d_Gval;
    int nGrow = 0;
    DevBuf d_sub_R, d_sub_dof_ptr, d_sub_dofs, d_sub_region, d_sub_Sbase, d_g2l, d_weights;
    DevBuf d_sub_ker, d_sub_Gcol, d_sub_Abase, d_sub_nlocal, d_pair_sub, d_pair_k, d_acc, d_lam1, d_lam2, d_wsum;
    DevBuf d_unit_of_dk, d_dnlocal, d_dAbase, d_cell_out, d_edge_out, d_sAbase, d_u_out, d_p_out;
    DevBuf d_mom;  // p1 p2 u1 u2 for moments output
    DevBuf d_flag; // index validation flag
    // CG workspace
    DevBuf w_slot_q, w_init;   // CG slot -> batch position; slots to start
    DevBuf w_r, w_p, w_rr, w_r0, w_pend, w_iters, w_relres, w_status, w_active, w_any, w_alpha, w_Slam;
    int64_t w_cap = 0;
    // realization groups (grouped operator), one set per CG lane; the moment
    // passes use the first
    Groups grp[kMaxLanes];
    // host tables of the allocation-free CG (its device tables live in the scratch array)
    Groups grp_noalloc;
    std::vector<int> noalloc_ident, noalloc_sel;
    std::vector<int32_t> noalloc_act;
    DevBuf d_part, d_pos, w_Y;
    std::vector<int64_t> h_gidx;
    int64_t SR = 0;
    // tuning options (sdmm_set_option)
    int64_t opt_chunk = 0;   // realizations per CG chunk, 0 = from the cache budget
    int opt_check = 64;      // iterations between convergence checks
    int opt_graph = 1;       // capture the iteration group in a HIP graph
    int opt_basis_launch = 0;   // Darcy basis layout: 0 tuned, 1 one launch per shape class, 2 one queue
    // exact-mass units whose face-pressure band does not fit the LDS window:
    // the first n_wide entries of h_order, built in chunks through the tiled
    // band LDL^T (one StokesDev per unit, offsets into the chunk buffers)
    int n_wide = 0;
    std::vector<WideChunk> wide_chunks;
    int64_t wt_cap_tiles = 0, wt_cap_rhs = 0, wt_cap_linv = 0;   // doubles of the chunk buffers
    DevBuf d_wide_sdx, d_wide_units, d_wt_tiles, d_wt_tilesN, d_wt_linv, d_wt_rhs, d_wt_tmp;
    int basis_mode[2] = {0, 0};  // layout the tuner picked per precision (FP64, mixed); 0: not tuned yet
    int queue_rs[2] = {0, 0};    // solve group width of the one-queue layout per precision
    int opt_ktime = 0;       // 0: no kernel timing; n: time one iteration of every n-th check group
    int opt_stokes_rebuild = 0;   // rebuild the Stokes basis on every build_flux_basis
    int opt_stokes_refine = 0;    // FP64 refinement steps of the Stokes solves
    bool moments_final = false;   // the field moments in d_mom match the accumulators
    std::vector<hipEvent_t> kev;   // event pool of the kernel timing
    hipStream_t cap_stream = nullptr;
    hipStream_t stokes_cap = nullptr;        // capture stream of the Stokes graph
    hipStream_t stokes_side = nullptr;       // second stream of the Stokes factor (the rest updates)
    hipStream_t stokes_fwd = nullptr;        // third: the forward sweep of the first solve, beside the factor
    hipStream_t stokes_run = nullptr;        // the Stokes build runs here, beside the Darcy build
    hipEvent_t stokes_ev[6] = {};            // panel done, the rest updates of four columns, forward sweep done
    hipGraph_t stokes_graph = nullptr;
    hipGraphExec_t stokes_exec = nullptr;
    hipStream_t lane_stream = nullptr;   // the second CG lane
    hipEvent_t lane_ev = nullptr;        // the second lane starts after the work queued before it
    int opt_lanes = 2;                   // CG lanes (1 or 2)
    int32_t* h_count = nullptr;          // pinned: per lane the active count and the timed count
    std::map<int64_t, std::unique_ptr<CgStream>> streams;   // CG streams (continuous batching)
    const BasisView* view = nullptr;     // the basis the CG and moments use (null: stochastic)
    DetBatch det;                        // Method S2
    int64_t next_stream = 1;
    sdmm_counters counters{};
    hipEvent_t ev[9] = {};   // 0-2 build, 3-4 solve, 5 caller fork, 6-7 moments, 8 Stokes build done
    bool moments_timed = false;
};

namespace {

int fail(Prob* c, int code, const std::string& msg) {
    if (c) c->err = msg;
    return code;
}

#define HIPCHK(call)                                                                        \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(ctx, SDMM_EDEVICE, std::string(#call ": ") + hipGetErrorString(e_)); \
    } while (0)

int alloc(Prob* ctx, DevBuf& b, size_t bytes) {
    b.release();
    if (bytes == 0) bytes = 8;
    if (ctx->alloc) {
        b.p = ctx->alloc->alloc(bytes, ctx->device, ctx->alloc->user);
        if (!b.p) return fail(ctx, SDMM_ENOMEM, "the allocator gave no " + std::to_string(bytes) + " bytes");
        b.al = ctx->alloc;
        b.dev = ctx->device;
    } else {
        hipError_t e = hipMalloc(&b.p, bytes);
        if (e != hipSuccess) {
            b.p = nullptr;
            return fail(ctx, SDMM_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
        }
    }
    b.bytes = bytes;
    return SDMM_OK;
}

template <class T>
int upload(Prob* ctx, DevBuf& b, const std::vector<T>& v) {
    int rc = alloc(ctx, b, v.size() * sizeof(T));
    if (rc) return rc;
    if (!v.empty()) HIPCHK(hipMemcpy(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return SDMM_OK;
}

// The same on stream st (then waited for): ordered after the work queued on
// st, and no operation on the null stream, which HIP refuses while another
// thread captures a graph (a Method S2 batch laid out beside a serving
// engine's captured CG).
template <class T>
int upload_on(Prob* ctx, DevBuf& b, const std::vector<T>& v, hipStream_t st) {
    int rc = alloc(ctx, b, v.size() * sizeof(T));
    if (rc) return rc;
    if (!v.empty()) {
        HIPCHK(hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
    }
    return SDMM_OK;
}

DarcyTables darcy_tables(Prob* c) {
    DarcyTables t;
    t.dar = c->d_dar.as<DarcyDev>();
    t.units = c->d_units.as<UnitDev>();
    t.be_cell = c->d_be_cell.as<int>();
    t.be_kind = c->d_be_kind.as<int>();
    t.be_len = c->d_be_len.as<double>();
    t.be_hperp = c->d_be_hperp.as<double>();
    t.be_medge = c->d_be_medge.as<int>();
    t.be_sgn = c->d_be_sgn.as<int>();
    t.cell_be = c->d_cell_be.as<int>();
    t.Pi = c->d_Pi.as<double>();
    t.phi = c->d_phi.as<double>();
    t.xi = c->d_xi.as<double>();
    t.supp_ptr = c->d_supp_ptr.as<int>();
    t.supp_e = c->d_supp_e.as<int>();
    t.supp_v = c->d_supp_v.as<double>();
    t.me_cell = c->d_me_cell.as<int>();
    t.order = c->d_order.as<int>();
    t.unit_base = 0;
    return t;
}

// T scratch of one unit: K, the transmissibilities and the mortar-edge
// terms (5-point operator), or K and the five band diagonals of the padded
// face-pressure system (exact mass)
static int64_t darcy_tscr(const DarcyHost& h) {
    return h.exact ? (int64_t)h.N + 5LL * ((h.Ns + 15) / 16 * 16) : 4LL * h.N + h.n_medge;
}

// Chunks of wide units (ids into `units`, in order): each chunk within
// the given doubles of tiles (twice: L and the backward tiles), right-hand
// sides (twice: solution and scratch) and inverses, or, with no caps (0),
// within about 4 GB of all of them; one StokesDev per unit with its offsets
// into the chunk buffers.
void plan_wide(const Problem& P, const std::vector<UnitDev>& units, const std::vector<int>& ids, int64_t cap_t,
               int64_t cap_r, int64_t cap_l, std::vector<WideChunk>& chunks, std::vector<StokesDev>& sdx) {
    chunks.clear();
    sdx.clear();
    WideChunk ch{};
    auto close_chunk = [&]() {
        if (ch.count > 0) chunks.push_back(ch);
        ch = WideChunk{};
        ch.first = (int)sdx.size();
    };
    close_chunk();
    for (int u : ids) {
        const DarcyHost& h = P.darcy[units[u].d];
        StokesDev x{};
        x.nband = h.Ns;
        x.nblk = (h.Ns + 63) / 64;
        x.w = (h.bs + 63) / 64;
        x.ncol = h.R;
        x.R = h.R;
        const int64_t nt = (int64_t)x.nblk * (x.w + 1) * 4096, nr = (int64_t)x.nblk * 64 * x.ncol,
                      nl = (int64_t)x.nblk * 4096;
        const bool full = cap_t > 0 ? (ch.tiles + nt > cap_t || ch.rhs + nr > cap_r || ch.linv + nl > cap_l)
                                    : (2 * (ch.tiles + nt) + ch.linv + nl + 2 * (ch.rhs + nr)) * 8 > (int64_t)4 << 30;
        if (ch.count > 0 && full) close_chunk();
        x.off_tiles = ch.tiles;
        x.off_rhs = ch.rhs;
        x.off_linv = ch.linv;
        ch.tiles += nt;
        ch.rhs += nr;
        ch.linv += nl;
        ch.count++;
        ch.max_nblk = std::max(ch.max_nblk, x.nblk);
        ch.max_w = std::max(ch.max_w, x.w);
        ch.max_ncol = std::max(ch.max_ncol, x.ncol);
        ch.max_ld = std::max(ch.max_ld, x.nblk * 64);
        ch.max_np = std::max(ch.max_np, (h.Ns + 15) / 16 * 16);
        sdx.push_back(x);
    }
    close_chunk();
}

int setup_device(Prob* ctx) {
    Problem& P = ctx->P;
    const int nsub = (int)P.subs.size();
    // ---- Darcy tables and units
    std::vector<DarcyDev> dar;
    std::vector<int> be_cell, be_kind, be_medge, be_sgn, cell_be, supp_ptr, supp_e, me_cell;
    std::vector<double> be_len, be_hperp, Pi, phi, supp_v;
    std::vector<double> xi;
    std::vector<int64_t> region_xi_off(P.n_region);
    for (int r = 0; r < P.n_region; ++r) {
        region_xi_off[r] = (int64_t)xi.size();
        for (int k = 0; k < P.nlocal[r]; ++k)
            for (int s = 0; s < P.region_nterm[r]; ++s)
                xi.push_back(P.node_x[P.local_ids[r][(size_t)k * P.region_nterm[r] + s]]);
    }
    if (xi.empty()) xi.push_back(0.0);
    ctx->units.clear();
    ctx->sub_Sbase.assign(nsub, 0);
    ctx->sub_R.assign(nsub, 0);
    ctx->sub_region.assign(nsub, -1);
    ctx->sub_ker.assign(nsub, 0);
    ctx->sub_Gcol.assign(nsub, 0);
    ctx->sub_nlocal.assign(nsub, 1);
    ctx->sub_Abase.assign(nsub, 0);
    int64_t S_off = 0, X_off = 0, L_off = 0, T_off = 0, A_off = 0, I_off = 0;
    ctx->max_b = 0;
    ctx->max_R = 0;
    ctx->max_Rd = 0;
    ctx->max_nout_d = 0;
    ctx->max_units_per_d = 0;
    ctx->cell_out_off.clear();
    ctx->edge_out_off.clear();
    int64_t cell_tot = 0, edge_tot = 0;
    std::vector<int> unit_of_dk, dnlocal;
    std::vector<int64_t> dAbase;
    for (size_t di = 0; di < P.darcy.size(); ++di)
        ctx->max_units_per_d = std::max(ctx->max_units_per_d, P.nlocal[P.subs[P.darcy[di].sub].region]);
    for (size_t di = 0; di < P.darcy.size(); ++di) {
        const DarcyHost& h = P.darcy[di];
        DarcyDev d{};
        d.nx = h.nx;
        d.ny = h.ny;
        d.N = h.N;
        d.swap = h.swap;
        d.b = h.b;
        d.exact = h.exact;
        d.Ns = h.Ns;
        d.bs = h.bs;
        d.R = h.R;
        d.nterm = h.nterm;
        d.n_medge = h.n_medge;
        d.hx = h.hx;
        d.hy = h.hy;
        d.nu = P.in.nu_d;
        d.mean_logk = h.mean_logk;
        d.off_be = (int64_t)be_cell.size();
        d.off_cellbe = (int64_t)cell_be.size();
        d.off_Pi = (int64_t)Pi.size();
        d.off_phi = (int64_t)phi.size();
        d.off_dofs = P.sub_ptr[h.sub];
        d.off_supp = (int64_t)supp_ptr.size();
        d.off_me = (int64_t)me_cell.size();
        be_cell.insert(be_cell.end(), h.be_cell.begin(), h.be_cell.end());
        be_kind.insert(be_kind.end(), h.be_kind.begin(), h.be_kind.end());
        be_medge.insert(be_medge.end(), h.be_medge.begin(), h.be_medge.end());
        be_sgn.insert(be_sgn.end(), h.be_sgn.begin(), h.be_sgn.end());
        be_len.insert(be_len.end(), h.be_len.begin(), h.be_len.end());
        be_hperp.insert(be_hperp.end(), h.be_hperp.begin(), h.be_hperp.end());
        Pi.insert(Pi.end(), h.Pi.begin(), h.Pi.end());
        phi.resize(phi.size() + (size_t)h.nterm * h.N);   // filled on the device (launch_kl)
        std::vector<int> cb((size_t)2 * h.N, -1);
        me_cell.resize(me_cell.size() + h.n_medge);
        for (size_t e = 0; e < h.be_cell.size(); ++e) {
            int c = h.be_cell[e];
            if (cb[2 * c] < 0) cb[2 * c] = (int)e;
            else cb[2 * c + 1] = (int)e;
            if (h.be_medge[e] >= 0) {
                int ci = h.swap ? (c % h.nx) * h.ny + c / h.nx : c;
                me_cell[d.off_me + h.be_medge[e]] = ci;
            }
        }
        cell_be.insert(cell_be.end(), cb.begin(), cb.end());
        // support lists: for every mortar DOF, the mortar edges where its average is non-zero
        int base = (int)supp_e.size();
        std::vector<std::vector<std::pair<int, double>>> sl(h.R);
        for (int e = 0; e < h.n_medge; ++e)
            for (int m = 0; m < h.R; ++m) {
                double v = h.Pi[(size_t)e * h.R + m];
                if (v != 0.0) sl[m].push_back({e, v});
            }
        for (int m = 0; m < h.R; ++m) {
            supp_ptr.push_back(base);
            for (auto& pr : sl[m]) {
                supp_e.push_back(pr.first);
                supp_v.push_back(pr.second);
                ++base;
            }
        }
        supp_ptr.push_back(base);
        dar.push_back(d);
        const int i = h.sub;
        const int r = P.subs[i].region;
        ctx->sub_R[i] = h.R;
        ctx->sub_region[i] = r;
        ctx->sub_nlocal[i] = P.nlocal[r];
        ctx->sub_Sbase[i] = S_off;
        ctx->sub_Abase[i] = A_off;
        dAbase.push_back(A_off);
        dnlocal.push_back(P.nlocal[r]);
        for (int k = 0; k < ctx->max_units_per_d; ++k) unit_of_dk.push_back(k < P.nlocal[r] ? (int)ctx->units.size() + k : -1);
        for (int k = 0; k < P.nlocal[r]; ++k) {
            UnitDev u{};
            u.d = (int)di;
            u.k = k;
            u.sub = i;
            u.off_xi = region_xi_off[r] + (int64_t)k * P.region_nterm[r];
            u.off_S = S_off;
            u.off_X = X_off;
            u.off_L = L_off;
            u.off_T = T_off;
            u.off_I = I_off;
            // the blocked factor pads rows to a multiple of 16 and the band to bp
            const int64_t Np = (h.Ns + 15) / 16 * 16, bp = (h.bs + 15) / 16 * 16;
            S_off += (int64_t)h.R * h.R;
            X_off += Np * h.R;
            L_off += Np * (bp + 1);
            I_off += Np * 16;
            T_off += darcy_tscr(h);
            A_off += (int64_t)h.R + (int64_t)h.R * h.R;
            ctx->units.push_back(u);
            ctx->pair_sub.push_back(i);
            ctx->pair_k.push_back(k);
        }
        ctx->max_b = std::max(ctx->max_b, h.bs);
        ctx->max_R = std::max(ctx->max_R, h.R);
        ctx->max_Rd = std::max(ctx->max_Rd, h.R);
        int nout = h.N + (h.nx + 1) * h.ny + h.nx * (h.ny + 1);
        ctx->max_nout_d = std::max(ctx->max_nout_d, nout);
        ctx->cell_out_off.push_back(cell_tot);
        ctx->edge_out_off.push_back(edge_tot);
        cell_tot += h.N;
        edge_tot += (int64_t)(h.nx + 1) * h.ny + (int64_t)h.nx * (h.ny + 1);
    }
    ctx->n_units = (int64_t)ctx->units.size();
    {
        // shape classes, most expensive unit shape first; units whose band
        // does not fit the LDS window (only the exact mass has them) first of all
        std::map<std::pair<int, int>, std::vector<int>> cls;
        for (size_t u = 0; u < ctx->units.size(); ++u) {
            const DarcyHost& h = P.darcy[ctx->units[u].d];
            cls[{(h.bs + 15) / 16 * 16, (h.R + 3) & ~3}].push_back((int)u);
        }
        std::vector<std::pair<double, std::pair<int, int>>> rank;
        for (auto& kv : cls) {
            const DarcyHost& h = P.darcy[ctx->units[kv.second[0]].d];
            const double cost = (double)h.Ns * kv.first.first * (kv.first.first + kv.first.second);
            rank.push_back({(kv.first.first > kMaxDarcyBand ? -1e300 : 0.0) - cost, kv.first});
        }
        std::sort(rank.begin(), rank.end());
        ctx->classes.clear();
        ctx->h_order.clear();
        ctx->n_wide = 0;
        ctx->max_b = 0;
        for (auto& rk : rank) {
            const auto& ids = cls[rk.second];
            if (rk.second.first > kMaxDarcyBand) {
                ctx->h_order.insert(ctx->h_order.end(), ids.begin(), ids.end());
                ctx->n_wide += (int)ids.size();
                continue;
            }
            int np = 0;
            for (int u : ids) np = std::max(np, (P.darcy[ctx->units[u].d].Ns + 15) / 16 * 16);
            ctx->classes.push_back(
                {(int)ctx->h_order.size(), (int)ids.size(), rk.second.first, rk.second.second, np, {0, 0}});
            ctx->h_order.insert(ctx->h_order.end(), ids.begin(), ids.end());
            ctx->max_b = std::max(ctx->max_b, rk.second.first);
        }
    }
    // the block kernels hold a band block of 16 (bp + 1) <= 8 x 256 values in
    // registers and index band columns below 128: bp <= 112 for every unit
    // that runs through the LDS window
    if (ctx->max_b > kMaxDarcyBand || darcy_factor_lds(ctx->max_b, 8) > 150 * 1024 ||
        darcy_solve_lds(ctx->max_b, ctx->max_Rd, 8) > 150 * 1024)
        return fail(ctx, SDMM_EINVAL, "a Darcy subdomain's band window does not fit (shorter side above 112 cells)");
    {
        // chunks of the wide units, each within about 4 GB of tiles, inverses
        // and right-hand sides
        std::vector<StokesDev> sdx;
        std::vector<int> wunits(ctx->h_order.begin(), ctx->h_order.begin() + ctx->n_wide);
        plan_wide(P, ctx->units, wunits, 0, 0, 0, ctx->wide_chunks, sdx);
        int64_t mt = 0, mr = 0, ml = 0;
        for (auto& c : ctx->wide_chunks) {
            mt = std::max(mt, c.tiles);
            mr = std::max(mr, c.rhs);
            ml = std::max(ml, c.linv);
        }
        ctx->wt_cap_tiles = mt;
        ctx->wt_cap_rhs = mr;
        ctx->wt_cap_linv = ml;
        int rc;
        if (ctx->n_wide > 0 && !ctx->host_only) {
            if ((rc = upload(ctx, ctx->d_wide_sdx, sdx)) || (rc = upload(ctx, ctx->d_wide_units, wunits)) ||
                (rc = alloc(ctx, ctx->d_wt_tiles, mt * 8)) || (rc = alloc(ctx, ctx->d_wt_tilesN, mt * 8)) ||
                (rc = alloc(ctx, ctx->d_wt_linv, ml * 8)) || (rc = alloc(ctx, ctx->d_wt_rhs, mr * 8)) ||
                (rc = alloc(ctx, ctx->d_wt_tmp, mr * 8)))
                return rc;
        }
    }
    // ---- Stokes
    ctx->sdev.clear();
    std::vector<int> tr_sub, tr_r, tr_c, bmap, q_ptr, q_col;
    std::vector<double> tr_v, Zc, q_val, uD;
    std::vector<int64_t> uD_off;
    int64_t tiles_off = 0, rhs_off = 0, U_off = 0, P_off = 0, linv_off = 0;
    int gcol = 0;
    ctx->max_nblk = ctx->max_w = ctx->max_ncol = 0;
    ctx->max_nout_s = 0;
    ctx->u_out_off.clear();
    ctx->p_out_off.clear();
    int64_t u_tot = 0, p_tot = 0;
    std::vector<int64_t> sAbase;
    for (size_t si = 0; si < P.stokes.size(); ++si) {
        const StokesHost& h = P.stokes[si];
        StokesDev s{};
        s.nband = h.nband;
        s.nblk = (h.nband + 63) / 64;
        s.w = (h.bw + 63) / 64;
        s.ncol = h.R + 1;
        s.nvel = h.nvel;
        s.npre = h.npre;
        s.R = h.R;
        s.nker = h.nker;
        s.off_tiles = tiles_off;
        s.off_rhs = rhs_off;
        s.off_U = U_off;
        s.off_P = P_off;
        s.off_map = (int64_t)bmap.size();
        s.off_Z = (int64_t)Zc.size();
        s.off_q = (int64_t)q_ptr.size();
        s.off_S = S_off;
        s.off_dofs = P.sub_ptr[h.sub];
        s.off_G = gcol;
        s.off_linv = linv_off;
        linv_off += (int64_t)s.nblk * 4096;
        tiles_off += (int64_t)s.nblk * (s.w + 1) * 4096;
        rhs_off += (int64_t)s.nblk * 64 * s.ncol;
        U_off += (int64_t)s.nvel * s.ncol;
        P_off += (int64_t)s.npre * s.ncol;
        for (int q = 0; q < h.nband; ++q) bmap.push_back(h.band_kind[q] == 0 ? h.band_raw[q] : -1 - h.band_raw[q]);
        Zc.insert(Zc.end(), h.Z.begin(), h.Z.end());
        int qb = (int)q_col.size();
        for (int m = 0; m <= h.R; ++m) q_ptr.push_back(qb + h.q_ptr[m]);
        q_col.insert(q_col.end(), h.q_col.begin(), h.q_col.end());
        q_val.insert(q_val.end(), h.q_val.begin(), h.q_val.end());
        uD_off.push_back((int64_t)uD.size());
        uD.insert(uD.end(), h.uD.begin(), h.uD.end());
        for (size_t q = 0; q < h.ar.size(); ++q) {
            tr_sub.push_back((int)si);
            tr_r.push_back(h.ar[q]);
            tr_c.push_back(h.ac[q]);
            tr_v.push_back(h.av[q]);
        }
        const int i = h.sub;
        ctx->sub_R[i] = h.R;
        ctx->sub_region[i] = -1;
        ctx->sub_ker[i] = h.nker;
        ctx->sub_Gcol[i] = gcol;
        ctx->sub_nlocal[i] = 1;
        ctx->sub_Sbase[i] = S_off;
        ctx->sub_Abase[i] = A_off;
        sAbase.push_back(A_off);
        const int ext = h.R + h.nker;
        A_off += (int64_t)ext + (int64_t)ext * ext;
        S_off += (int64_t)h.R * h.R;
        gcol += h.nker;
        ctx->pair_sub.push_back(i);
        ctx->pair_k.push_back(0);
        ctx->sdev.push_back(s);
        ctx->max_nblk = std::max(ctx->max_nblk, s.nblk);
        ctx->max_w = std::max(ctx->max_w, s.w);
        ctx->max_ncol = std::max(ctx->max_ncol, s.ncol);
        ctx->max_R = std::max(ctx->max_R, h.R);
        ctx->max_nout_s = std::max(ctx->max_nout_s, h.nvel + h.npre);
        ctx->u_out_off.push_back(u_tot);
        ctx->p_out_off.push_back(p_tot);
        u_tot += h.nvel;
        p_tot += h.npre;
    }
    ctx->max_ext = 0;
    for (int i = 0; i < nsub; ++i) ctx->max_ext = std::max(ctx->max_ext, ctx->sub_R[i] + ctx->sub_ker[i]);
    if ((size_t)64 * ctx->max_ext * 8 > 150 * 1024) return fail(ctx, SDMM_EINVAL, "too many mortar DOFs on one subdomain");
    if (P.n_kernel > 16) return fail(ctx, SDMM_EINVAL, "more than 16 FETI kernel modes");
    if (P.M > 256 * 8) return fail(ctx, SDMM_EINVAL, "more than 2048 mortar DOFs");
    if ((size_t)(64 * (ctx->max_R + 1) + 64 * ctx->max_R) * 8 > 160 * 1024)
        return fail(ctx, SDMM_EINVAL, "too many mortar DOFs on one subdomain for the grouped operator");
    ctx->n_trip = (int64_t)tr_v.size();
    ctx->S_total = S_off;
    ctx->X_total = X_off;
    ctx->L_total = L_off;
    ctx->I_total = I_off;
    ctx->T_total = T_off;
    ctx->A_total = A_off;
    ctx->field_size[0] = P.M;
    ctx->field_size[1] = cell_tot;
    ctx->field_size[2] = edge_tot;
    ctx->field_size[3] = u_tot;
    ctx->field_size[4] = p_tot;
    if (ctx->host_only) return SDMM_OK;
    // ---- uploads
    int rc;
#define UP(buf, vec) \
    if ((rc = upload(ctx, buf, vec))) return rc;
    UP(ctx->d_dar, dar);
    UP(ctx->d_units, ctx->units);
    UP(ctx->d_order, ctx->h_order);
    UP(ctx->d_be_cell, be_cell);
    UP(ctx->d_be_kind, be_kind);
    UP(ctx->d_be_len, be_len);
    UP(ctx->d_be_hperp, be_hperp);
    UP(ctx->d_be_medge, be_medge);
    UP(ctx->d_be_sgn, be_sgn);
    UP(ctx->d_cell_be, cell_be);
    UP(ctx->d_Pi, Pi);
    {
        // the KL modes and the phi tables on the device (the kept modes and
        // eigenvalues come back to the problem, for sdmm_get_kl)
        std::vector<KLRegionDev> kreg;
        int nm_max = 1, nt_max = 1, max_cells = 0;
        for (int r = 0; r < P.n_region; ++r) {
            const double* rr = &P.region_rect[4 * r];
            KLRegionDev k{};
            k.ax = 0.5 * (rr[1] - rr[0]);
            k.ay = 0.5 * (rr[3] - rr[2]);
            k.etax = P.region_eta[2 * r];
            k.etay = P.region_eta[2 * r + 1];
            k.sigma2 = P.region_sigma2[r];
            k.xc = 0.5 * (rr[0] + rr[1]);
            k.yc = 0.5 * (rr[2] + rr[3]);
            k.nterm = P.region_nterm[r];
            k.nm = k.nterm + 1;
            nm_max = std::max(nm_max, k.nm);
            nt_max = std::max(nt_max, k.nterm);
            kreg.push_back(k);
        }
        std::vector<KLSubDev> ksub;
        for (size_t di = 0; di < P.darcy.size(); ++di) {
            const Sub& sb = P.subs[P.darcy[di].sub];
            KLSubDev q{};
            q.x0 = sb.x0;
            q.y0 = sb.y0;
            q.hx = sb.hx;
            q.hy = sb.hy;
            q.nx = sb.nx;
            q.ny = sb.ny;
            q.region = sb.region;
            q.off_phi = dar[di].off_phi;
            max_cells = std::max(max_cells, sb.nx * sb.ny);
            ksub.push_back(q);
        }
        DevBuf d_kreg, d_ksub, d_w, d_nrm, d_lam1, d_ma, d_mb, d_lam2;
        const size_t nr = std::max(1, P.n_region);
        if ((rc = upload(ctx, d_kreg, kreg)) || (rc = upload(ctx, d_ksub, ksub)) ||
            (rc = alloc(ctx, d_w, nr * 2 * nm_max * 8)) || (rc = alloc(ctx, d_nrm, nr * 2 * nm_max * 8)) ||
            (rc = alloc(ctx, d_lam1, nr * 2 * nm_max * 8)) || (rc = alloc(ctx, d_ma, nr * nt_max * 4)) ||
            (rc = alloc(ctx, d_mb, nr * nt_max * 4)) || (rc = alloc(ctx, d_lam2, nr * nt_max * 8)) ||
            (rc = alloc(ctx, ctx->d_phi, std::max<size_t>(phi.size(), 1) * 8)))
            return rc;
        HIPCHK(launch_kl(d_kreg.as<KLRegionDev>(), P.n_region, d_ksub.as<KLSubDev>(), (int)ksub.size(), nm_max, nt_max,
                         max_cells, d_w.as<double>(), d_nrm.as<double>(), d_lam1.as<double>(), d_ma.as<int>(),
                         d_mb.as<int>(), d_lam2.as<double>(), ctx->d_phi.as<double>(), nullptr));
        std::vector<int> hma(nr * nt_max), hmb(nr * nt_max);
        std::vector<double> hl(nr * nt_max);
        HIPCHK(hipMemcpy(hma.data(), d_ma.p, hma.size() * 4, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(hmb.data(), d_mb.p, hmb.size() * 4, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(hl.data(), d_lam2.p, hl.size() * 8, hipMemcpyDeviceToHost));
        for (int r = 0; r < P.n_region; ++r)
            for (int t = 0; t < P.region_nterm[r]; ++t) {
                P.kl[r].ma[t] = hma[r * nt_max + t];
                P.kl[r].mb[t] = hmb[r * nt_max + t];
                P.kl[r].lam[t] = hl[r * nt_max + t];
            }
    }
    UP(ctx->d_xi, xi);
    UP(ctx->d_supp_ptr, supp_ptr);
    UP(ctx->d_supp_e, supp_e);
    UP(ctx->d_supp_v, supp_v);
    UP(ctx->d_me_cell, me_cell);
    UP(ctx->d_sdev, ctx->sdev);
    UP(ctx->d_bmap, bmap);
    UP(ctx->d_Z, Zc);
    UP(ctx->d_q_ptr, q_ptr);
    UP(ctx->d_q_col, q_col);
    UP(ctx->d_q_val, q_val);
    UP(ctx->d_uD, uD);
    UP(ctx->d_uD_off, uD_off);
    UP(ctx->d_tr_sub, tr_sub);
    UP(ctx->d_tr_r, tr_r);
    UP(ctx->d_tr_c, tr_c);
    UP(ctx->d_tr_v, tr_v);
    std::vector<int64_t> dofs(P.sub_dofs.begin(), P.sub_dofs.end());
    UP(ctx->d_sub_dofs, dofs);
    UP(ctx->d_sub_dof_ptr, P.sub_ptr);
    {
        // the two subdomain-local positions of every mortar DOF, lower subdomain first
        std::vector<int> pos((size_t)2 * P.M, -1);
        for (size_t q = 0; q < P.sub_dofs.size(); ++q) {
            const int64_t m = P.sub_dofs[q];
            if (pos[2 * m] < 0) pos[2 * m] = (int)q;
            else if (pos[2 * m + 1] < 0) pos[2 * m + 1] = (int)q;
            else return fail(ctx, SDMM_EINVAL, "a mortar DOF belongs to more than two subdomains");
        }
        for (int m = 0; m < P.M; ++m)
            if (pos[2 * m + 1] < 0) return fail(ctx, SDMM_EINVAL, "a mortar DOF belongs to one subdomain only");
        UP(ctx->d_pos, pos);
        ctx->SR = P.sub_ptr[nsub];
    }
    UP(ctx->d_sub_R, ctx->sub_R);
    UP(ctx->d_sub_region, ctx->sub_region);
    UP(ctx->d_sub_Sbase, ctx->sub_Sbase);
    UP(ctx->d_sub_ker, ctx->sub_ker);
    UP(ctx->d_sub_Gcol, ctx->sub_Gcol);
    UP(ctx->d_sub_Abase, ctx->sub_Abase);
    UP(ctx->d_sub_nlocal, ctx->sub_nlocal);
    UP(ctx->d_pair_sub, ctx->pair_sub);
    UP(ctx->d_pair_k, ctx->pair_k);
    UP(ctx->d_g2l, P.g2l);
    UP(ctx->d_weights, P.weights);
    UP(ctx->d_unit_of_dk, unit_of_dk);
    UP(ctx->d_dnlocal, dnlocal);
    UP(ctx->d_dAbase, dAbase);
    UP(ctx->d_cell_out, ctx->cell_out_off);
    UP(ctx->d_edge_out, ctx->edge_out_off);
    UP(ctx->d_sAbase, sAbase);
    UP(ctx->d_u_out, ctx->u_out_off);
    UP(ctx->d_p_out, ctx->p_out_off);
#undef UP
    if ((rc = alloc(ctx, ctx->d_S, ctx->S_total * 8))) return rc;
    if ((rc = alloc(ctx, ctx->d_X, ctx->X_total * 8))) return rc;
    if ((rc = alloc(ctx, ctx->d_L, ctx->L_total * 8))) return rc;
    if ((rc = alloc(ctx, ctx->d_I, std::max<int64_t>(ctx->I_total, 1) * 8))) return rc;
    if ((rc = alloc(ctx, ctx->d_T, ctx->T_total * 8))) return rc;
    if ((rc = alloc(ctx, ctx->d_tiles, tiles_off * 8))) return rc;
    if ((rc = alloc(ctx, ctx->d_tiles0, tiles_off * 8))) return rc;
    if ((rc = alloc(ctx, ctx->d_tilesN, tiles_off * 8))) return rc;
    if ((rc = alloc(ctx, ctx->d_linv, linv_off * 8))) return rc;
    if ((rc = alloc(ctx, ctx->d_stmp, rhs_off * 8))) return rc;
    if ((rc = alloc(ctx, ctx->d_rhs, rhs_off * 8))) return rc;
    if ((rc = alloc(ctx, ctx->d_U, U_off * 8))) return rc;
    if ((rc = alloc(ctx, ctx->d_P, P_off * 8))) return rc;
    if ((rc = alloc(ctx, ctx->d_g, (size_t)P.M * 8))) return rc;
    if ((rc = alloc(ctx, ctx->d_G, (size_t)P.M * std::max(1, P.n_kernel) * 8))) return rc;
    if ((rc = alloc(ctx, ctx->d_GtGinv, (size_t)std::max(1, P.n_kernel * P.n_kernel) * 8))) return rc;
    if ((rc = alloc(ctx, ctx->d_acc, ctx->A_total * 8))) return rc;
    if ((rc = alloc(ctx, ctx->d_lam1, (size_t)P.M * 8))) return rc;
    if ((rc = alloc(ctx, ctx->d_lam2, (size_t)P.M * 8))) return rc;
    if ((rc = alloc(ctx, ctx->d_wsum, 8))) return rc;
    if ((rc = alloc(ctx, ctx->d_refine, 16))) return rc;
    if ((rc = alloc(ctx, ctx->d_flag, 8))) return rc;
    int64_t mom = 2 * (ctx->field_size[1] + ctx->field_size[2] + ctx->field_size[3] + ctx->field_size[4]);
    if ((rc = alloc(ctx, ctx->d_mom, (size_t)std::max<int64_t>(mom, 1) * 8))) return rc;
    // Stokes RHS into the padded band layout
    std::vector<double> rhs((size_t)rhs_off, 0.0);
    for (size_t si = 0; si < P.stokes.size(); ++si) {
        const StokesHost& h = P.stokes[si];
        const StokesDev& s = ctx->sdev[si];
        const int64_t ld = (int64_t)s.nblk * 64;
        for (int c = 0; c < s.ncol; ++c)
            for (int q = 0; q < h.nband; ++q) rhs[s.off_rhs + c * ld + q] = h.rhs[(size_t)c * h.nband + q];
    }
    ctx->d_rhs.release();
    if ((rc = upload(ctx, ctx->d_rhs, rhs))) return rc;
    ctx->d_rhs0.release();
    if ((rc = upload(ctx, ctx->d_rhs0, rhs))) return rc;
    if ((rc = alloc(ctx, ctx->d_res, std::max<size_t>(rhs.size(), 1) * 8))) return rc;
    HIPCHK(hipMemset(ctx->d_acc.p, 0, ctx->d_acc.bytes));
    HIPCHK(hipMemset(ctx->d_lam1.p, 0, ctx->d_lam1.bytes));
    HIPCHK(hipMemset(ctx->d_lam2.p, 0, ctx->d_lam2.bytes));
    HIPCHK(hipMemset(ctx->d_wsum.p, 0, 8));
    return SDMM_OK;
}

// The device part of the Stokes build (Section 5.1, eqs. starSproblem1-2 and
// barSproblem1-2 for every Stokes subdomain): assembly into tiles, the band
// LDL^T (on st and a second stream), the sweep tiles, the solves for all
// R + 1 right-hand sides with the optional FP64 refinement steps, and the
// traces that give S, g_H and G.  Only kernels, device copies and event
// waits, so the whole sequence can be captured as one graph.
int stokes_device_work(Prob* ctx, hipStream_t st) {
    Problem& P = ctx->P;
    const int ns = (int)ctx->sdev.size();
    HIPCHK(launch_fill_zero(ctx->d_g.as<double>(), (int64_t)(ctx->d_g.bytes / 8), st));
    HIPCHK(launch_fill_zero(ctx->d_G.as<double>(), (int64_t)(ctx->d_G.bytes / 8), st));
    if (ns == 0) return SDMM_OK;
    StokesDev* sd = ctx->d_sdev.as<StokesDev>();
    double* tiles = ctx->d_tiles.as<double>();
    double* x = ctx->d_rhs.as<double>();
    double* res = ctx->d_res.as<double>();
    const double* linv = ctx->d_linv.as<double>();
    // the right-hand sides are solved in place: start from the stored ones
    HIPCHK(hipMemcpyAsync(ctx->d_rhs.p, ctx->d_rhs0.p, ctx->d_rhs.bytes, hipMemcpyDeviceToDevice, st));
    HIPCHK(launch_fill_zero(tiles, (int64_t)(ctx->d_tiles.bytes / 8), st));
    HIPCHK(launch_stokes_scatter(sd, ns, ctx->d_tr_sub.as<int>(), ctx->d_tr_r.as<int>(), ctx->d_tr_c.as<int>(),
                                 ctx->d_tr_v.as<double>(), ctx->n_trip, tiles, st));
    HIPCHK(launch_stokes_pad_identity(sd, ns, ctx->max_nblk, tiles, st));
    // the assembled matrix, kept for the refinement residuals
    if (ctx->opt_stokes_refine > 0)
        HIPCHK(hipMemcpyAsync(ctx->d_tiles0.p, ctx->d_tiles.p, ctx->d_tiles.bytes, hipMemcpyDeviceToDevice, st));
    // the factor, block column by block column: diag and panel of column J on
    // st; the rest updates of column J on the side stream, which the diag
    // launch of column J + 2 waits for (every tile still receives its updates
    // in increasing J); the forward step J of the first solve on a third
    // stream, as soon as L(., J) is final
    hipStream_t side = ctx->stokes_side, fwd = ctx->stokes_fwd;
    hipEvent_t* ev = ctx->stokes_ev;
    for (int J = 0; J < ctx->max_nblk; ++J) {
        if (J >= 2) HIPCHK(hipStreamWaitEvent(st, ev[1 + (J - 2) % 4], 0));
        HIPCHK(launch_stokes_ldl_diag(sd, ns, J, tiles, ctx->d_linv.as<double>(), st));
        HIPCHK(launch_stokes_ldl_panel(sd, ns, J, ctx->max_w, tiles, linv, st));
        HIPCHK(hipEventRecord(ev[0], st));
        HIPCHK(hipStreamWaitEvent(side, ev[0], 0));
        HIPCHK(hipStreamWaitEvent(fwd, ev[0], 0));
        HIPCHK(launch_stokes_ldl_rest(sd, ns, J, ctx->max_w, tiles, side));
        HIPCHK(hipEventRecord(ev[1 + J % 4], side));
        HIPCHK(launch_stokes_fwd_early(sd, ns, J, ctx->max_w, ctx->max_ncol, tiles, linv, x,
                                       ctx->d_stmp.as<double>(), fwd));
        HIPCHK(launch_stokes_sweep_row(sd, ns, J, ctx->max_w, tiles, ctx->d_tilesN.as<double>(), linv, fwd));
    }
    HIPCHK(hipEventRecord(ev[5], fwd));
    // join the side stream (the last columns' rest updates) and the third
    // one (forward sweep, backward sweep tiles); the refinement solves need
    // the forward sweep tiles M in place of L as well
    for (int J = std::max(0, ctx->max_nblk - 2); J < ctx->max_nblk; ++J)
        HIPCHK(hipStreamWaitEvent(st, ev[1 + J % 4], 0));
    HIPCHK(hipStreamWaitEvent(st, ev[5], 0));
    if (ctx->opt_stokes_refine > 0)
        HIPCHK(launch_stokes_sweep_tiles(sd, ns, ctx->max_nblk, ctx->max_w, tiles, ctx->d_tilesN.as<double>(), linv,
                                         st));
    auto solve = [&](double* b) {
        return launch_stokes_solve(sd, ns, ctx->max_nblk, ctx->max_w, ctx->max_ncol, tiles, ctx->d_tilesN.as<double>(),
                                   linv, b, ctx->d_stmp.as<double>(), st);
    };
    // the first solve: its forward sweep ran beside the factor
    HIPCHK(launch_stokes_solve_back(sd, ns, ctx->max_nblk, ctx->max_w, ctx->max_ncol, tiles,
                                    ctx->d_tilesN.as<double>(), linv, x, ctx->d_stmp.as<double>(), st));
    // optional FP64 iterative refinement against the assembled matrix
    for (int step = 0; step < ctx->opt_stokes_refine; ++step) {
        HIPCHK(launch_stokes_residual(sd, ns, ctx->max_nblk, ctx->max_ncol, ctx->d_tiles0.as<double>(),
                                      ctx->d_rhs0.as<double>(), x, res, st));
        HIPCHK(solve(res));
        HIPCHK(launch_add_inplace(x, res, (int64_t)(ctx->d_rhs.bytes / 8), st));
    }
    HIPCHK(launch_stokes_finish(sd, ns, ctx->max_ncol, ctx->max_R, ctx->d_rhs.as<double>(), ctx->d_bmap.as<int>(),
                                ctx->d_uD.as<double>(), ctx->d_uD_off.as<int64_t>(), ctx->d_Z.as<double>(),
                                ctx->d_q_ptr.as<int>(), ctx->d_q_col.as<int>(), ctx->d_q_val.as<double>(),
                                ctx->d_sub_dofs.as<int64_t>(), ctx->d_U.as<double>(), ctx->d_P.as<double>(),
                                ctx->d_S.as<double>(), ctx->d_g.as<double>(), ctx->d_G.as<double>(), P.M, st));
    return SDMM_OK;
}

int build_stokes(Prob* ctx, hipStream_t st) {
    Problem& P = ctx->P;
    if (!ctx->stokes_side) {
        if (hipStreamCreateWithFlags(&ctx->stokes_side, hipStreamNonBlocking) != hipSuccess) {
            ctx->stokes_side = nullptr;
            return fail(ctx, SDMM_EDEVICE, "second stream of the Stokes factor");
        }
        if (hipStreamCreateWithFlags(&ctx->stokes_fwd, hipStreamNonBlocking) != hipSuccess) {
            ctx->stokes_fwd = nullptr;
            return fail(ctx, SDMM_EDEVICE, "third stream of the Stokes factor");
        }
        for (hipEvent_t& e : ctx->stokes_ev)
            if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
                e = nullptr;
                return fail(ctx, SDMM_EDEVICE, "events of the Stokes factor");
            }
    }
    if (!ctx->opt_graph) {
        int rc = stokes_device_work(ctx, st);
        if (rc) return rc;
    } else {
        // about 3,000 small launches on two streams per build: captured once
        // as a graph and replayed on every later build of this problem
        if (!ctx->stokes_exec) {
            if (!ctx->stokes_cap && hipStreamCreateWithFlags(&ctx->stokes_cap, hipStreamNonBlocking) != hipSuccess) {
                ctx->stokes_cap = nullptr;
                return fail(ctx, SDMM_EDEVICE, "stream for the Stokes graph");
            }
            HIPCHK(hipStreamBeginCapture(ctx->stokes_cap, hipStreamCaptureModeThreadLocal));
            int rc = stokes_device_work(ctx, ctx->stokes_cap);
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamEndCapture(ctx->stokes_cap, &g);
            if (rc) {
                if (g) (void)hipGraphDestroy(g);
                return rc;
            }
            if (e != hipSuccess || !g) return fail(ctx, SDMM_EDEVICE, "capture of the Stokes build failed");
            if (hipGraphInstantiate(&ctx->stokes_exec, g, nullptr, nullptr, 0) != hipSuccess) {
                (void)hipGraphDestroy(g);
                ctx->stokes_exec = nullptr;
                return fail(ctx, SDMM_EDEVICE, "instantiation of the Stokes graph failed");
            }
            ctx->stokes_graph = g;
        }
        HIPCHK(hipGraphLaunch(ctx->stokes_exec, st));
    }
    // FETI coarse matrix (G^T G)^{-1}: n_kernel x n_kernel, inverted on the host
    const int nk = P.n_kernel;
    if (nk > 0) {
        std::vector<double> G((size_t)P.M * nk);
        HIPCHK(hipMemcpyAsync(G.data(), ctx->d_G.p, G.size() * 8, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        std::vector<double> A((size_t)nk * nk), Inv((size_t)nk * nk, 0.0);
        for (int a = 0; a < nk; ++a)
            for (int b = 0; b < nk; ++b) {
                double s = 0;
                for (int m = 0; m < P.M; ++m) s += G[(size_t)a * P.M + m] * G[(size_t)b * P.M + m];
                A[a * nk + b] = s;
            }
        for (int a = 0; a < nk; ++a) Inv[a * nk + a] = 1.0;
        for (int c = 0; c < nk; ++c) {  // Gauss-Jordan with partial pivoting
            int piv = c;
            for (int r = c + 1; r < nk; ++r)
                if (std::fabs(A[r * nk + c]) > std::fabs(A[piv * nk + c])) piv = r;
            if (std::fabs(A[piv * nk + c]) < 1e-300) return fail(ctx, SDMM_EINVAL, "singular FETI coarse matrix");
            for (int k = 0; k < nk; ++k) {
                std::swap(A[c * nk + k], A[piv * nk + k]);
                std::swap(Inv[c * nk + k], Inv[piv * nk + k]);
            }
            double d = A[c * nk + c];
            for (int k = 0; k < nk; ++k) {
                A[c * nk + k] /= d;
                Inv[c * nk + k] /= d;
            }
            for (int r = 0; r < nk; ++r)
                if (r != c) {
                    double f = A[r * nk + c];
                    for (int k = 0; k < nk; ++k) {
                        A[r * nk + k] -= f * A[c * nk + k];
                        Inv[r * nk + k] -= f * Inv[c * nk + k];
                    }
                }
        }
        HIPCHK(hipMemcpy(ctx->d_GtGinv.p, Inv.data(), Inv.size() * 8, hipMemcpyHostToDevice));
        // rows of G that are not zero (the mortar DOFs of floating subdomains)
        std::vector<int> rows;
        std::vector<double> vals;
        for (int m = 0; m < P.M; ++m) {
            bool nz = false;
            for (int k = 0; k < nk; ++k) nz |= G[(size_t)k * P.M + m] != 0.0;
            if (!nz) continue;
            rows.push_back(m);
            for (int k = 0; k < nk; ++k) vals.push_back(G[(size_t)k * P.M + m]);
        }
        int rc;
        if ((rc = upload(ctx, ctx->d_Grow, rows))) return rc;
        if ((rc = upload(ctx, ctx->d_Gval, vals))) return rc;
        ctx->nGrow = (int)rows.size();
    }
    return SDMM_OK;
}

CgArgs cg_args(Prob* ctx, int64_t n, const int64_t* gidx, double* lam) {
    CgArgs a{};
    a.n = n;
    a.M = ctx->P.M;
    a.nsub = (int)ctx->P.subs.size();
    a.nregion = ctx->P.n_region;
    a.nker = ctx->P.n_kernel;
    a.gidx = gidx;
    a.g2l = ctx->d_g2l.as<int32_t>();
    a.sub_R = ctx->d_sub_R.as<int>();
    a.sub_dof_ptr = ctx->d_sub_dof_ptr.as<int64_t>();
    a.sub_dofs = ctx->d_sub_dofs.as<int64_t>();
    a.sub_region = ctx->d_sub_region.as<int>();
    a.sub_Sbase = ctx->view ? ctx->view->d_sub_Sbase.as<int64_t>() : ctx->d_sub_Sbase.as<int64_t>();
    a.S_cache = ctx->view ? ctx->view->S : ctx->d_S.as<double>();
    a.g = ctx->d_g.as<double>();
    a.G = ctx->d_G.as<double>();
    a.GtGinv = ctx->d_GtGinv.as<double>();
    a.lam = lam;
    a.r = ctx->w_r.as<double>();
    a.p = ctx->w_p.as<double>();
    a.rr = ctx->w_rr.as<double>();
    a.r0 = ctx->w_r0.as<double>();
    a.pend = ctx->w_pend.as<double>();
    a.iters = ctx->w_iters.as<int32_t>();
    a.relres = ctx->w_relres.as<double>();
    a.status = ctx->w_status.as<int32_t>();
    a.active = ctx->w_active.as<int32_t>();
    a.any_active = ctx->w_any.as<int32_t>();
    a.Grow = ctx->d_Grow.as<int>();
    a.Gval = ctx->d_Gval.as<double>();
    a.nGrow = ctx->nGrow;
    return a;
}

// Every global index must address a collocation point; checked on the
// device before any kernel dereferences the global->local table.
int check_indices(Prob* ctx, const int64_t* gidx, int64_t n, hipStream_t st) {
    int32_t bad = 0;
    HIPCHK(hipMemsetAsync(ctx->d_flag.p, 0, 4, st));
    HIPCHK(launch_validate_index(gidx, n, ctx->P.nreal, ctx->d_flag.as<int32_t>(), st));
    HIPCHK(hipMemcpyAsync(&bad, ctx->d_flag.p, 4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (bad) return fail(ctx, SDMM_EINVAL, "a global collocation index is out of range");
    return SDMM_OK;
}

// Sort the batch by local realization index, region by region, and cut the
// (subdomain, local realization) groups into chunks of at most 64
// realizations (moment work items) and 64 rows of S (operator work items).
int fetch_gidx(Prob* ctx, const int64_t* gidx, int64_t n, hipStream_t st) {
    ctx->h_gidx.resize(n);
    HIPCHK(hipMemcpyAsync(ctx->h_gidx.data(), gidx, n * 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return SDMM_OK;
}

// The host tables of the realization groups.  subset: positions of the
// realizations to include (null means all n); hg: host global index of every
// position.
int build_groups_host(Prob* ctx, Groups& G, int64_t n, const std::vector<int>* subset, const int64_t* hg) {
    const Problem& P = ctx->P;
    std::vector<int> all;
    if (!subset) {
        all.resize(n);
        for (int64_t l = 0; l < n; ++l) all[l] = (int)l;
        subset = &all;
    }
    const std::vector<int>& sel = *subset;
    n = (int64_t)sel.size();
    G.h_perm.clear();
    G.h_work.clear();
    G.h_awork.clear();
    G.h_slot.clear();
    G.h_item0.clear();
    const int nr = P.n_region;
    const BasisView* v = ctx->view;
    const int32_t* g2l = v ? v->g2l.data() : P.g2l.data();
    const std::vector<int>& nloc = v ? v->nlocal : P.nlocal;
    const std::vector<int>& pair_sub = v ? v->pair_sub : ctx->pair_sub;
    const std::vector<int>& pair_k = v ? v->pair_k : ctx->pair_k;
    std::vector<int64_t> rbase(nr + 1);
    std::vector<std::vector<int64_t>> goff(nr);
    for (int r = 0; r < nr; ++r) {
        rbase[r] = (int64_t)G.h_perm.size();
        const int L = nloc[r];
        goff[r].assign(L + 1, 0);
        for (int64_t q = 0; q < n; ++q) goff[r][g2l[(size_t)hg[sel[q]] * nr + r] + 1]++;
        for (int k = 0; k < L; ++k) goff[r][k + 1] += goff[r][k];
        std::vector<int64_t> fill(goff[r].begin(), goff[r].end() - 1);
        G.h_perm.resize(G.h_perm.size() + n);
        for (int64_t q = 0; q < n; ++q) {
            const int k = g2l[(size_t)hg[sel[q]] * nr + r];
            G.h_perm[rbase[r] + fill[k]++] = sel[q];
        }
    }
    rbase[nr] = (int64_t)G.h_perm.size();
    for (int64_t q = 0; q < n; ++q) G.h_perm.push_back(sel[q]);  // Stokes: every realization
    if ((int64_t)G.h_perm.size() > 2147483647LL) return fail(ctx, SDMM_EINVAL, "batch too large");
    int64_t slot = 0;
    for (size_t pidx = 0; pidx < pair_sub.size(); ++pidx) {
        const int i = pair_sub[pidx], k = pair_k[pidx];
        const int R = ctx->sub_R[i];
        const int r = ctx->sub_region[i];
        const int ext = R + ctx->sub_ker[i];
        const int64_t g0 = r >= 0 ? goff[r][k] : 0, g1 = r >= 0 ? goff[r][k + 1] : n;
        const int64_t base = r >= 0 ? rbase[r] : rbase[nr];
        G.h_item0.push_back((int)G.h_awork.size());
        // product items: the row blocks of a chunk of realizations sit kXcds
        // items apart, so that they run on one XCD and its L2 serves the
        // chunk's coefficients to every row block
        for (int64_t cb = g0; cb < g1; cb += 64 * kXcds)
            for (int row0 = 0; row0 < R; row0 += 64)
                for (int64_t c0 = cb; c0 < std::min<int64_t>(g1, cb + 64 * kXcds); c0 += 64) {
                    const int cnt = (int)std::min<int64_t>(64, g1 - c0);
                    G.h_work.push_back(make_int4(i, k, row0 | (cnt << 16), (int)(base + c0)));
                }
        for (int64_t c0 = g0; c0 < g1; c0 += 64) {
            const int cnt = (int)std::min<int64_t>(64, g1 - c0);
            G.h_awork.push_back(make_int4(i, k, cnt, (int)(base + c0)));
            G.h_slot.push_back(slot);
            slot += (int64_t)ext + (int64_t)ext * ext;
        }
    }
    G.h_item0.push_back((int)G.h_awork.size());
    G.nwork = (int)G.h_work.size();
    G.nawork = (int)G.h_awork.size();
    G.part_total = slot;
    return SDMM_OK;
}

// The group tables to the device (buffers grown as needed).
int upload_groups(Prob* ctx, Groups& G, hipStream_t st) {
    int rc;
    auto grow = [&](DevBuf& b, size_t bytes) { return b.bytes < bytes ? alloc(ctx, b, bytes) : SDMM_OK; };
    if ((rc = grow(G.d_perm, G.h_perm.size() * 4))) return rc;
    if ((rc = grow(G.d_work, G.h_work.size() * 16))) return rc;
    if ((rc = grow(G.d_awork, G.h_awork.size() * 16))) return rc;
    if ((rc = grow(G.d_slot, G.h_slot.size() * 8))) return rc;
    if ((rc = grow(G.d_item0, G.h_item0.size() * 4))) return rc;
    HIPCHK(hipMemcpyAsync(G.d_perm.p, G.h_perm.data(), G.h_perm.size() * 4, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(G.d_work.p, G.h_work.data(), G.h_work.size() * 16, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(G.d_awork.p, G.h_awork.data(), G.h_awork.size() * 16, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(G.d_slot.p, G.h_slot.data(), G.h_slot.size() * 8, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(G.d_item0.p, G.h_item0.data(), G.h_item0.size() * 4, hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));  // the host vectors are reused by the next chunk
    return SDMM_OK;
}

int build_groups(Prob* ctx, Groups& G, int64_t n, const std::vector<int>* subset, const int64_t* hg,
                 hipStream_t st) {
    int rc = build_groups_host(ctx, G, n, subset, hg);
    return rc ? rc : upload_groups(ctx, G, st);
}

// Realizations in flight (CG slots, and the chunk of the moment passes): their
// vectors (lambda, r, p and the subdomain-local operator results) are kept
// within ~200 MB so that they stay resident in the 256 MB last-level cache
// between the product and the update.
int64_t chunk_size(Prob* ctx, int64_t n) {
    if (ctx->opt_chunk > 0) return std::min<int64_t>(n, ctx->opt_chunk);
    const int64_t per = (3 * (int64_t)ctx->P.M + ctx->SR) * 8 + 64;
    const int64_t c = std::max<int64_t>(256, (int64_t)(200.0 * 1024 * 1024) / per);
    return std::min(n, c);
}

int ensure_workspace(Prob* ctx, int64_t n) {
    if (n <= ctx->w_cap) return SDMM_OK;
    const size_t M = ctx->P.M;
    int rc;
    if ((rc = alloc(ctx, ctx->w_r, n * M * 8))) return rc;
    if ((rc = alloc(ctx, ctx->w_p, n * M * 8))) return rc;
    if ((rc = alloc(ctx, ctx->w_Slam, n * M * 8))) return rc;
    if ((rc = alloc(ctx, ctx->w_rr, n * 8))) return rc;
    if ((rc = alloc(ctx, ctx->w_r0, n * 8))) return rc;
    if ((rc = alloc(ctx, ctx->w_pend, n * 8))) return rc;
    if ((rc = alloc(ctx, ctx->w_iters, n * 4))) return rc;
    if ((rc = alloc(ctx, ctx->w_relres, n * 8))) return rc;
    if ((rc = alloc(ctx, ctx->w_status, n * 4))) return rc;
    if ((rc = alloc(ctx, ctx->w_active, n * 4))) return rc;
    if ((rc = alloc(ctx, ctx->w_any, 8 * kMaxLanes))) return rc;   // per lane: active count, timed count
    if ((rc = alloc(ctx, ctx->w_alpha, n * std::max(1, ctx->P.n_kernel) * 8))) return rc;
    if ((rc = alloc(ctx, ctx->w_Y, (size_t)n * ctx->SR * 8))) return rc;
    if ((rc = alloc(ctx, ctx->w_slot_q, n * 4))) return rc;
    if ((rc = alloc(ctx, ctx->w_init, n * 4))) return rc;
    ctx->w_cap = n;
    return SDMM_OK;
}

}  // namespace

namespace {

// One launch per shape class, each on its own stream (forked from and joined
// back into `st`), largest class first; a single class runs on `st` itself.
template <class F>
hipError_t launch_classes(Prob* ctx, hipStream_t st, F&& launch) {
    DarcyTables t = darcy_tables(ctx);
    const int nc = (int)ctx->classes.size();
    if (nc == 1) {
        const auto& c = ctx->classes[0];
        t.unit_base = c.base;
        return launch(t, c, st);
    }
    const int ns = std::min(nc, 4);
    hipError_t e;
    while ((int)ctx->class_streams.size() < ns) {
        hipStream_t q = nullptr;
        if ((e = hipStreamCreateWithFlags(&q, hipStreamNonBlocking)) != hipSuccess) return e;
        ctx->class_streams.push_back(q);
    }
    while ((int)ctx->class_events.size() < ns + 1) {
        hipEvent_t ev = nullptr;
        if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess) return e;
        ctx->class_events.push_back(ev);
    }
    if ((e = hipEventRecord(ctx->class_events[ns], st)) != hipSuccess) return e;
    for (int q = 0; q < ns; ++q)
        if ((e = hipStreamWaitEvent(ctx->class_streams[q], ctx->class_events[ns], 0)) != hipSuccess) return e;
    for (int c = 0; c < nc; ++c) {
        const auto& cl = ctx->classes[c];
        t.unit_base = cl.base;
        if ((e = launch(t, cl, ctx->class_streams[c % ns])) != hipSuccess) return e;
    }
    for (int q = 0; q < ns; ++q) {
        if ((e = hipEventRecord(ctx->class_events[q], ctx->class_streams[q])) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(st, ctx->class_events[q], 0)) != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

namespace {

// A new problem slot on the context's device (device -1: host only).
int impl_create(int device, const sdmm_alloc* al, Prob** out) {
    *out = nullptr;
    Prob* c = new (std::nothrow) Prob();
    if (!c) return SDMM_ENOMEM;
    c->device = device;
    c->alloc = al;
    if (device == -1) {
        c->host_only = true;
        *out = c;
        return SDMM_OK;
    }
    if (hipSetDevice(device) != hipSuccess) {
        delete c;
        return SDMM_EDEVICE;
    }
    for (auto& e : c->ev)
        if (hipEventCreate(&e) != hipSuccess) {
            delete c;
            return SDMM_EDEVICE;
        }
    *out = c;
    return SDMM_OK;
}

int impl_destroy(Prob* ctx) {
    if (!ctx) return SDMM_EINVAL;
    if (ctx->host_only) {
        delete ctx;
        return SDMM_OK;
    }
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    if (ctx->stokes_exec) (void)hipGraphExecDestroy(ctx->stokes_exec);
    if (ctx->stokes_graph) (void)hipGraphDestroy(ctx->stokes_graph);
    if (ctx->stokes_cap) (void)hipStreamDestroy(ctx->stokes_cap);
    if (ctx->stokes_side) (void)hipStreamDestroy(ctx->stokes_side);
    if (ctx->stokes_fwd) (void)hipStreamDestroy(ctx->stokes_fwd);
    if (ctx->stokes_run) (void)hipStreamDestroy(ctx->stokes_run);
    for (hipEvent_t e : ctx->stokes_ev)
        if (e) (void)hipEventDestroy(e);
    if (ctx->lane_stream) (void)hipStreamDestroy(ctx->lane_stream);
    if (ctx->h_count) (void)hipHostFree(ctx->h_count);
    if (ctx->lane_ev) (void)hipEventDestroy(ctx->lane_ev);
    for (auto& e : ctx->ev)
        if (e) (void)hipEventDestroy(e);
    for (auto& e : ctx->kev)
        if (e) (void)hipEventDestroy(e);
    for (auto& e : ctx->class_events)
        if (e) (void)hipEventDestroy(e);
    for (auto& q : ctx->class_streams)
        if (q) (void)hipStreamDestroy(q);
    delete ctx;
    return SDMM_OK;
}


int impl_set_problem(Prob* ctx, const sdmm_problem* p) {
    if (!ctx->host_only) {
        HIPCHK(hipSetDevice(ctx->device));
        HIPCHK(hipDeviceSynchronize());
    }
    ctx->have_problem = false;
    ctx->basis_built = false;
    ctx->stokes_built = false;
    std::string err = build_problem(*p, ctx->P);
    if (!err.empty()) return fail(ctx, SDMM_EINVAL, err);
    ctx->w_cap = 0;
    ctx->pair_sub.clear();
    ctx->pair_k.clear();
    int rc = setup_device(ctx);
    if (rc) return rc;
    ctx->counters = sdmm_counters{};
    ctx->have_problem = true;
    return SDMM_OK;
}

int impl_get_sizes(Prob* ctx, sdmm_sizes* o) {
    if (!ctx || !o) return fail(ctx, SDMM_EINVAL, "null argument");
    if (!ctx->have_problem) return fail(ctx, SDMM_ESTATE, "no problem set");
    const Problem& P = ctx->P;
    *o = sdmm_sizes{};
    o->n_sub = (int64_t)P.subs.size();
    o->n_stokes = P.n_stokes;
    o->n_darcy = P.n_darcy;
    o->n_iface = (int64_t)P.ifaces.size();
    o->M = P.M;
    o->n_real = P.nreal;
    o->n_term = P.nterm;
    o->n_region = P.n_region;
    o->n_units = ctx->n_units;
    int nf = 0;
    for (auto& s : P.stokes) nf += s.floating;
    o->n_floating = nf;
    o->n_kernel = P.n_kernel;
    for (int k = 0; k < 5; ++k) o->field_size[k] = ctx->field_size[k];
    o->basis_bytes = ctx->S_total * 8;
    o->response_bytes = ctx->X_total * 8;
    o->max_R = ctx->max_R;
    int64_t fl = 0;
    for (auto& u : ctx->units) {
        const DarcyHost& h = P.darcy[u.d];
        fl += (int64_t)h.Ns * h.bs * h.bs + 4LL * h.Ns * h.bs * h.R;
    }
    o->darcy_flops = fl;
    return SDMM_OK;
}

int impl_get_index_map(Prob* ctx, int kind, int64_t* out, int64_t cap, int64_t* n_out) {
    if (!ctx || !n_out) return fail(ctx, SDMM_EINVAL, "null argument");
    if (!ctx->have_problem) return fail(ctx, SDMM_ESTATE, "no problem set");
    const Problem& P = ctx->P;
    std::vector<int64_t> v;
    switch (kind) {
        case SDMM_MAP_INTERFACES:
            for (auto& f : P.ifaces) {
                v.push_back(f.i);
                v.push_back(f.j);
                v.push_back(f.kind);
                v.push_back(f.ndof);
                v.push_back(f.off);
            }
            break;
        case SDMM_MAP_SUB_PTR: v.assign(P.sub_ptr.begin(), P.sub_ptr.end()); break;
        case SDMM_MAP_SUB_DOFS: v.assign(P.sub_dofs.begin(), P.sub_dofs.end()); break;
        case SDMM_MAP_SUB_SIGN: v.assign(P.sub_sign.begin(), P.sub_sign.end()); break;
        case SDMM_MAP_G2L: v.assign(P.g2l.begin(), P.g2l.end()); break;
        case SDMM_MAP_NLOCAL: v.assign(P.nlocal.begin(), P.nlocal.end()); break;
        case SDMM_MAP_NODE_IDS: v.assign(P.ids.begin(), P.ids.end()); break;
        default: return fail(ctx, SDMM_EINVAL, "unknown map kind");
    }
    *n_out = (int64_t)v.size();
    if (!out) return SDMM_OK;
    if (cap < (int64_t)v.size()) return fail(ctx, SDMM_EINVAL, "output capacity too small");
    std::copy(v.begin(), v.end(), out);
    return SDMM_OK;
}

int impl_get_collocation(Prob* ctx, double* points, double* weights) {
    if (!ctx) return SDMM_EINVAL;
    if (!ctx->have_problem) return fail(ctx, SDMM_ESTATE, "no problem set");
    const Problem& P = ctx->P;
    if (points)
        for (size_t q = 0; q < P.ids.size(); ++q) points[q] = P.node_x[P.ids[q]];
    if (weights) std::copy(P.weights.begin(), P.weights.end(), weights);
    return SDMM_OK;
}

int impl_get_kl(Prob* ctx, int region, double* lam, int32_t* modes) {
    if (!ctx) return SDMM_EINVAL;
    if (!ctx->have_problem) return fail(ctx, SDMM_ESTATE, "no problem set");
    if (region < 0 || region >= ctx->P.n_region) return fail(ctx, SDMM_EINVAL, "bad region");
    const KLRegion& K = ctx->P.kl[region];
    for (size_t t = 0; t < K.lam.size(); ++t) {
        if (lam) lam[t] = K.lam[t];
        if (modes) {
            modes[2 * t] = K.ma[t];
            modes[2 * t + 1] = K.mb[t];
        }
    }
    return SDMM_OK;
}

// Mixed-precision refinement of the Darcy responses: corrections until the
// FP64 residual satisfies max|E - P X| <= kRefineTol max|E| per right-hand-
// side group, at most kMaxRefine of them.  The flux basis is then evaluated
// to second order in that residual (darcy_scorr_kernel), so its error is
// quadratic in kRefineTol; the responses themselves carry it linearly.
constexpr double kRefineTol = 1e-11;
constexpr int kMaxRefine = 4;

// The exact-mass units too wide for the LDS window, chunk by chunk (FP64):
// band and loads into zeroed tiles, identity on the padding rows, the band
// LDL^T block column by block column, the sweep tiles, the solve of all
// right-hand sides in place, then responses and flux bases.
// t: the unit tables (Method S3's, or a Method S2 batch's); chunks, d_sdx
// and d_units as planned by plan_wide; X, S and T the responses, bases and
// scratch the units' offsets point into.
int darcy_build_wide(Prob* ctx, const DarcyTables& t, const std::vector<WideChunk>& chunks, const DevBuf& d_sdx,
                     const DevBuf& d_units, double* X, double* S, double* T, hipStream_t st) {
    double* tiles = ctx->d_wt_tiles.as<double>();
    double* tilesN = ctx->d_wt_tilesN.as<double>();
    double* linv = ctx->d_wt_linv.as<double>();
    double* rhs = ctx->d_wt_rhs.as<double>();
    for (const auto& c : chunks) {
        const StokesDev* sdx = d_sdx.as<StokesDev>() + c.first;
        const int* units = d_units.as<int>() + c.first;
        HIPCHK(launch_fill_zero(tiles, c.tiles, st));
        HIPCHK(launch_fill_zero(rhs, c.rhs, st));
        HIPCHK(launch_exact_tiles_assemble(t, units, sdx, c.count, c.max_ld, tiles, rhs, T, st));
        HIPCHK(launch_stokes_pad_identity(sdx, c.count, c.max_nblk, tiles, st));
        for (int J = 0; J < c.max_nblk; ++J) {
            HIPCHK(launch_stokes_ldl_diag(sdx, c.count, J, tiles, linv, st));
            HIPCHK(launch_stokes_ldl_panel(sdx, c.count, J, c.max_w, tiles, linv, st));
            HIPCHK(launch_stokes_ldl_rest(sdx, c.count, J, c.max_w, tiles, st));
        }
        HIPCHK(launch_stokes_sweep_tiles(sdx, c.count, c.max_nblk, c.max_w, tiles, tilesN, linv, st));
        HIPCHK(launch_stokes_solve(sdx, c.count, c.max_nblk, c.max_w, c.max_ncol, tiles, tilesN, linv, rhs,
                                   ctx->d_wt_tmp.as<double>(), st));
        HIPCHK(launch_exact_tiles_finish(t, units, sdx, c.count, c.max_np, c.max_ncol, rhs, X, S, T, st));
    }
    return SDMM_OK;
}

// The Darcy units of a Method S3 build.  mode 1: one launch per shape class
// (LDS sized for the class) on forked streams, each class with its own solve
// group width; mode 2: one launch per phase over the whole queue of units,
// sorted by cost (largest shape first), LDS sized for the widest class.  The
// units too wide for the LDS window go first, through darcy_build_wide
// (skipped while the window layouts are timed).
int darcy_build(Prob* ctx, int precision, int mode, hipStream_t st, bool wide = true) {
    const int pi = precision == SDMM_PREC_MIXED ? 1 : 0;
    int rc;
    if (wide && ctx->n_wide > 0 &&
        (rc = darcy_build_wide(ctx, darcy_tables(ctx), ctx->wide_chunks, ctx->d_wide_sdx, ctx->d_wide_units,
                               ctx->d_X.as<double>(), ctx->d_S.as<double>(), ctx->d_T.as<double>(), st)))
        return rc;
    double* max_res = nullptr;
    int* steps = nullptr;
    if (pi == 1) {
        if (!ctx->d_L32.p && (rc = alloc(ctx, ctx->d_L32, ctx->L_total * 4))) return rc;
        if (!ctx->d_I32.p && (rc = alloc(ctx, ctx->d_I32, std::max<int64_t>(ctx->I_total, 1) * 4))) return rc;
        if (!ctx->d_W32.p && (rc = alloc(ctx, ctx->d_W32, ctx->X_total * 4))) return rc;
        if (!ctx->d_E.p && (rc = alloc(ctx, ctx->d_E, ctx->X_total * 8))) return rc;
        HIPCHK(hipMemsetAsync(ctx->d_refine.p, 0, 16, st));
        max_res = ctx->d_refine.as<double>();
        steps = reinterpret_cast<int*>(ctx->d_refine.as<char>() + 8);
    }
    auto launch = [&](const DarcyTables& tc, int count, int bp, int Rs, int np, int rs, hipStream_t q) {
        if (pi == 0)
            return launch_darcy_basis_blocked(tc, count, bp, Rs, np, rs, ctx->d_S.as<double>(), ctx->d_X.as<double>(),
                                              ctx->d_L.as<double>(), ctx->d_I.as<double>(), ctx->d_T.as<double>(),
                                              ctx->P.in.darcy_mass, q);
        return launch_darcy_basis_blocked_mixed(tc, count, bp, Rs, np, rs, ctx->d_S.as<double>(), ctx->d_X.as<double>(),
                                                ctx->d_E.as<double>(), ctx->d_L32.as<float>(), ctx->d_I32.as<float>(),
                                                ctx->d_T.as<double>(), ctx->d_W32.as<float>(), kMaxRefine, kRefineTol,
                                                max_res, steps, q);
    };
    if (ctx->classes.empty()) return SDMM_OK;
    if (mode == 2) {
        DarcyTables t = darcy_tables(ctx);
        t.unit_base = ctx->n_wide;
        int bp = 0, Rs = 0, np = 0;
        for (const auto& c : ctx->classes) {
            bp = std::max(bp, c.bp);
            Rs = std::max(Rs, c.Rs);
            np = std::max(np, c.np);
        }
        HIPCHK(launch(t, (int)ctx->n_units - ctx->n_wide, bp, Rs, np, ctx->queue_rs[pi], st));
    } else {
        HIPCHK(launch_classes(ctx, st, [&](const DarcyTables& tc, const Prob::UnitClass& c, hipStream_t q) {
            return launch(tc, c.count, c.bp, c.Rs, c.np, c.rs[pi], q);
        }));
    }
    return SDMM_OK;
}

// Tuning of the Darcy build at the first Method S3 build of a precision: every
// shape class alone with each solve group width that its right-hand sides
// need (16; 32 above 16; 64 above 32), the one-queue layout with each width,
// then both layouts with their best widths, each timed twice with events on
// the caller's stream (the smaller time counts); the fastest choices are kept
// for the builds that follow.  The results do not depend on them: every
// right-hand side is swept by the same per-column arithmetic.
int tune_darcy(Prob* ctx, int precision, hipStream_t st) {
    const int pi = precision == SDMM_PREC_MIXED ? 1 : 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(ctx, SDMM_EDEVICE, "events for the basis tuning");
    }
    int rc = SDMM_OK;
    auto timed = [&](auto&& run, double& ms) -> int {
        ms = 1e300;
        for (int rep = 0; rep < 2; ++rep) {
            int r;
            if (hipEventRecord(e0, st) != hipSuccess) return fail(ctx, SDMM_EDEVICE, "event record");
            if ((r = run())) return r;
            float t = 0.f;
            if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&t, e0, e1) != hipSuccess)
                return fail(ctx, SDMM_EDEVICE, "event timing");
            ms = std::min(ms, (double)t);
        }
        return SDMM_OK;
    };
    auto widths = [](int R) {
        std::vector<int> w{16};
        if (R > 16) w.push_back(32);
        if (R > 32) w.push_back(64);
        return w;
    };
    std::vector<Prob::UnitClass> saved = ctx->classes;
    const int nc = (int)ctx->classes.size();
    // classes one at a time: a build in the one-class layout of that class
    for (int c = 0; c < nc && !rc; ++c) {
        double best = 1e300;
        int best_w = 0;
        for (int w : widths(ctx->classes[c].Rs)) {
            std::vector<Prob::UnitClass> one{ctx->classes[c]};
            one[0].rs[pi] = w;
            std::swap(ctx->classes, one);
            double ms;
            rc = timed([&] { return darcy_build(ctx, precision, 1, st, false); }, ms);
            std::swap(ctx->classes, one);
            if (rc) break;
            if (ms < best) {
                best = ms;
                best_w = w;
            }
        }
        saved[c].rs[pi] = best_w;
    }
    ctx->classes = saved;
    int Rmax = 0;
    for (const auto& c : ctx->classes) Rmax = std::max(Rmax, c.Rs);
    double best_q = 1e300, per_class = 1e300;
    int best_qw = 0;
    for (int w : widths(Rmax)) {
        if (rc) break;
        ctx->queue_rs[pi] = w;
        double ms;
        if ((rc = timed([&] { return darcy_build(ctx, precision, 2, st, false); }, ms))) break;
        if (ms < best_q) {
            best_q = ms;
            best_qw = w;
        }
    }
    ctx->queue_rs[pi] = best_qw;
    if (!rc) rc = timed([&] { return darcy_build(ctx, precision, 1, st, false); }, per_class);
    ctx->basis_mode[pi] = rc ? 0 : (best_q < per_class ? 2 : 1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

int impl_build_flux_basis(Prob* ctx, int method, int precision, void* stream) {
    if (!ctx) return SDMM_EINVAL;
    if (ctx->host_only) return fail(ctx, SDMM_ESTATE, "context has no device");
    if (!ctx->have_problem) return fail(ctx, SDMM_ESTATE, "no problem set");
    if (precision != SDMM_PREC_FP64 && precision != SDMM_PREC_MIXED) return fail(ctx, SDMM_EINVAL, "bad precision");
    if (method != SDMM_METHOD_STOCHASTIC && method != SDMM_METHOD_DETERMINISTIC && method != SDMM_METHOD_PER_ITERATION)
        return fail(ctx, SDMM_EINVAL, "bad method");
    if (ctx->P.in.darcy_mass == 1 && (precision != SDMM_PREC_FP64 || method == SDMM_METHOD_PER_ITERATION))
        return fail(ctx, SDMM_EINVAL, "the exact RT0 mass is built in FP64 for Methods S2 and S3");
    HIPCHK(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    if (method == SDMM_METHOD_STOCHASTIC && ctx->opt_basis_launch == 0 &&
        ctx->basis_mode[precision == SDMM_PREC_MIXED ? 1 : 0] == 0) {
        int rc = tune_darcy(ctx, precision, st);
        if (rc) return rc;
    }
    HIPCHK(hipEventRecord(ctx->ev[0], st));
    ctx->method = method;
    ctx->det.valid = false;
    ctx->det.precision = precision;
    if (method != SDMM_METHOD_STOCHASTIC) {
        // Methods S2 and S1: the Darcy bases (S2) or factors (S1) are built per
        // batch inside solve_interface
    } else {
        const int pi = precision == SDMM_PREC_MIXED ? 1 : 0;
        int rc, mode = ctx->opt_basis_launch;
        if (mode == 0) mode = ctx->basis_mode[pi];
        if ((rc = darcy_build(ctx, precision, mode, st))) return rc;
    }
    HIPCHK(hipEventRecord(ctx->ev[1], st));
    if (!ctx->stokes_built || ctx->opt_stokes_rebuild) {
        // the Stokes build runs on its own stream from the start of the call,
        // beside the Darcy units queued on st (both are chains of small
        // dependent steps that leave most of the device idle)
        if (!ctx->stokes_run && hipStreamCreateWithFlags(&ctx->stokes_run, hipStreamNonBlocking) != hipSuccess) {
            ctx->stokes_run = nullptr;
            return fail(ctx, SDMM_EDEVICE, "stream for the Stokes build");
        }
        HIPCHK(hipStreamWaitEvent(ctx->stokes_run, ctx->ev[0], 0));
        int rc = build_stokes(ctx, ctx->stokes_run);
        if (rc) return rc;
        HIPCHK(hipEventRecord(ctx->ev[8], ctx->stokes_run));
        HIPCHK(hipStreamWaitEvent(st, ctx->ev[8], 0));
        ctx->stokes_built = true;
    } else {
        HIPCHK(hipEventRecord(ctx->ev[8], st));
    }
    HIPCHK(hipEventRecord(ctx->ev[2], st));
    ctx->built_precision = precision;
    ctx->basis_built = true;
    int64_t sd = 0, ss = 0;
    if (method == SDMM_METHOD_STOCHASTIC)
        for (auto& u : ctx->units) sd += ctx->P.darcy[u.d].R;
    for (auto& s : ctx->P.stokes) ss += s.R;
    ctx->counters.basis_solves_darcy += sd;
    ctx->counters.basis_solves_stokes = ss;
    ctx->counters.complementary_solves = (int64_t)ctx->P.stokes.size();
    if (method != SDMM_METHOD_STOCHASTIC) return SDMM_OK;
    ctx->counters.units_built += ctx->n_units;
    if (precision == SDMM_PREC_MIXED) {
        // every right-hand-side group must have reached the refinement tolerance
        double mr = 0.0;
        HIPCHK(hipMemcpyAsync(&mr, ctx->d_refine.p, 8, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (!(mr <= kRefineTol))
            return fail(ctx, SDMM_ENOTCONV,
                        "mixed-precision refinement stopped at relative residual " + std::to_string(mr) +
                            " above " + std::to_string(kRefineTol) + " (the basis is stored)");
    }
    return SDMM_OK;
}

int impl_get_basis(Prob* ctx, int sub, int k, double* S, int64_t ld) {
    if (!ctx || !S) return fail(ctx, SDMM_EINVAL, "null argument");
    if (!ctx->basis_built) return fail(ctx, SDMM_ESTATE, "basis not built");
    if (sub < 0 || sub >= (int)ctx->P.subs.size()) return fail(ctx, SDMM_EINVAL, "bad subdomain");
    const int R = ctx->sub_R[sub];
    if (ctx->method == SDMM_METHOD_PER_ITERATION && ctx->sub_region[sub] >= 0)
        return fail(ctx, SDMM_ESTATE, "Method S1 builds no Darcy basis");
    const bool det = ctx->method == SDMM_METHOD_DETERMINISTIC && ctx->sub_region[sub] >= 0;
    // Method S2: k is the batch position of the last solve
    const int64_t nk = det ? (ctx->det.valid ? ctx->det.n : 0) : ctx->sub_nlocal[sub];
    if (k < 0 || k >= nk || ld < R) return fail(ctx, SDMM_EINVAL, "bad local index or ld");
    HIPCHK(hipSetDevice(ctx->device));
    HIPCHK(hipDeviceSynchronize());
    std::vector<double> tmp((size_t)R * R);
    const double* src = ctx->d_S.as<double>() + ctx->sub_Sbase[sub] + (int64_t)k * R * R;
    if (det) {
        std::vector<int64_t> sb(ctx->P.subs.size());
        HIPCHK(hipMemcpy(sb.data(), ctx->det.view.d_sub_Sbase.p, sb.size() * 8, hipMemcpyDeviceToHost));
        src = ctx->det.d_S.as<double>() + sb[sub] + (int64_t)k * R * R;
    }
    HIPCHK(hipMemcpy(tmp.data(), src, tmp.size() * 8, hipMemcpyDeviceToHost));
    for (int j = 0; j < R; ++j)
        for (int m = 0; m < R; ++m) S[(int64_t)j * ld + m] = tmp[(size_t)j * R + m];
    return SDMM_OK;
}

int impl_get_interface_data(Prob* ctx, double* g, double* G) {
    if (!ctx) return SDMM_EINVAL;
    if (ctx->host_only) return fail(ctx, SDMM_ESTATE, "context has no device");
    if (!ctx->basis_built) return fail(ctx, SDMM_ESTATE, "basis not built");
    HIPCHK(hipSetDevice(ctx->device));
    HIPCHK(hipDeviceSynchronize());
    const size_t M = ctx->P.M;
    if (g) HIPCHK(hipMemcpy(g, ctx->d_g.p, M * 8, hipMemcpyDeviceToHost));
    if (G && ctx->P.n_kernel > 0) HIPCHK(hipMemcpy(G, ctx->d_G.p, (size_t)ctx->P.n_kernel * M * 8, hipMemcpyDeviceToHost));
    return SDMM_OK;
}

int impl_set_option(Prob* ctx, int option, int64_t value) {
    if (!ctx) return SDMM_EINVAL;
    switch (option) {
        case SDMM_OPT_CG_CHUNK:
            if (value < 0) return fail(ctx, SDMM_EINVAL, "chunk must be >= 0");
            ctx->opt_chunk = value;
            return SDMM_OK;
        case SDMM_OPT_CG_CHECK:
            if (value < 1 || value > 1024) return fail(ctx, SDMM_EINVAL, "check interval must be in 1..1024");
            ctx->opt_check = (int)value;
            return SDMM_OK;
        case SDMM_OPT_CG_GRAPH:
            ctx->opt_graph = value ? 1 : 0;
            return SDMM_OK;
        case SDMM_OPT_KERNEL_TIMING:
            if (value < 0 || value > 1 << 20) return fail(ctx, SDMM_EINVAL, "kernel timing period out of range");
            ctx->opt_ktime = (int)value;
            return SDMM_OK;
        case SDMM_OPT_STOKES_REBUILD:
            ctx->opt_stokes_rebuild = value ? 1 : 0;
            return SDMM_OK;
        case SDMM_OPT_STOKES_REFINE:
            if (value < 0 || value > 8) return fail(ctx, SDMM_EINVAL, "Stokes refinement steps must be in 0..8");
            if (value != ctx->opt_stokes_refine) {
                // the captured Stokes build holds the old step count
                if (ctx->stokes_exec) (void)hipGraphExecDestroy(ctx->stokes_exec);
                if (ctx->stokes_graph) (void)hipGraphDestroy(ctx->stokes_graph);
                ctx->stokes_exec = nullptr;
                ctx->stokes_graph = nullptr;
            }
            ctx->opt_stokes_refine = (int)value;
            return SDMM_OK;
        case SDMM_OPT_BASIS_LAUNCH:
            if (value < 0 || value > 2) return fail(ctx, SDMM_EINVAL, "basis launch layout must be 0, 1 or 2");
            ctx->opt_basis_launch = (int)value;
            return SDMM_OK;
        case SDMM_OPT_CG_LANES:
            if (value < 1 || value > kMaxLanes) return fail(ctx, SDMM_EINVAL, "cg_lanes must be 1 or 2");
            ctx->opt_lanes = (int)value;
            return SDMM_OK;
        default:
            return fail(ctx, SDMM_EINVAL, "unknown option");
    }
}

namespace {

// The batch through CG with S slots.  Slots are filled in batch order; when
// at least a sixteenth of a lane's slots hold finished realizations and some
// are still pending, the finished ones are retired (their iterations and
// status counted, their outputs already written by the kernels) and pending
// ones start in their place, so the operator keeps about S realizations in
// flight instead of draining once per chunk.  Once nothing is pending, a
// lane drops finished realizations from its operator when they are a quarter
// of its work.  With opt_lanes = 2 (and at least 2 kMinLaneSlots slots) the
// slots are split into two lanes with their own groups, graph and stream:
// the lanes' iterations are independent, so one lane's product (FP64 MFMA)
// overlaps the other's update (HBM) on the device.  A realization's
// arithmetic does not depend on its slot, lane or neighbours, so results do
// not depend on S or on the lanes.
constexpr int64_t kMinLaneSlots = 1024;   // smaller lanes gain nothing and cost latency

struct Lane {
    int id = 0;
    int64_t base = 0, S = 0;              // slots base .. base + S - 1 of the workspace
    hipStream_t s = nullptr;
    Groups* G = nullptr;
    CgArgs a{};
    double* Y = nullptr;
    std::vector<int> slot_q, init, sel;
    std::vector<int64_t> slot_g;          // global index of each slot's realization
    std::vector<int32_t> act, itv, stv;
    int64_t in_work = 0;                  // slots covered by the operator work list
    int64_t groups = 0;
    bool timed = false, done = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void release() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
    }
};

int solve_batch(Prob* ctx, int64_t n, int64_t S, const int64_t* gidx, double rtol, int32_t max_iter,
                double* lambda, int32_t* iters, double* relres, int32_t* status, hipStream_t st, int64_t& tot_it,
                bool& bad, bool& brk) {
    int rc;
    S = std::max<int64_t>(1, std::min(S, n));
    if ((rc = fetch_gidx(ctx, gidx, n, st))) return rc;
    int nl = (ctx->opt_lanes > 1 && S >= 2 * kMinLaneSlots) ? 2 : 1;
    if (nl == 2 && !ctx->lane_stream &&
        hipStreamCreateWithFlags(&ctx->lane_stream, hipStreamNonBlocking) != hipSuccess)
        ctx->lane_stream = nullptr;
    if (nl == 2 && !ctx->lane_ev && hipEventCreateWithFlags(&ctx->lane_ev, hipEventDisableTiming) != hipSuccess)
        ctx->lane_ev = nullptr;
    if (nl == 2 && (!ctx->lane_stream || !ctx->lane_ev)) nl = 1;
    // the active counts are read back into pinned memory, so queueing a lane's
    // read-back does not wait for its group
    if (!ctx->h_count && hipHostMalloc((void**)&ctx->h_count, 8 * kMaxLanes) != hipSuccess) {
        ctx->h_count = nullptr;
        return fail(ctx, SDMM_ENOMEM, "pinned host memory for the CG counts");
    }
    const int M = ctx->P.M;
    const int group = ctx->opt_check;
    const bool ktime = ctx->opt_ktime != 0;
    const int kTimeEvery = std::max(1, ctx->opt_ktime);   // one check group in kTimeEvery of lane 0 is timed
    Lane lanes[kMaxLanes];
    const CgArgs a0 = cg_args(ctx, S, gidx, lambda);
    for (int k = 0; k < nl; ++k) {
        Lane& L = lanes[k];
        L.id = k;
        L.base = k == 0 ? 0 : S / 2;
        L.S = nl == 1 ? S : (k == 0 ? S / 2 : S - S / 2);
        L.s = k == 0 ? st : ctx->lane_stream;
        L.G = &ctx->grp[k];
        CgArgs& a = L.a;
        a = a0;
        a.n = L.S;
        a.rtol = rtol;
        a.max_iter = max_iter;
        a.r += L.base * M;
        a.p += L.base * M;
        a.rr += L.base;
        a.r0 += L.base;
        a.pend += L.base;
        a.iters += L.base;
        a.relres += L.base;
        a.status += L.base;
        a.active += L.base;
        a.any_active += 2 * k;
        a.slot_q = ctx->w_slot_q.as<int>() + L.base;
        a.init_slots = ctx->w_init.as<int>() + L.base;
        a.iters_out = iters;
        a.relres_out = relres;
        a.status_out = status;
        L.Y = ctx->w_Y.as<double>() + L.base * ctx->SR;
        L.slot_q.assign(L.S, -1);
        L.slot_g.assign(L.S, 0);
        L.act.resize(L.S);
        L.itv.resize(L.S);
        L.stv.resize(L.S);
    }
    int64_t next = 0;   // next batch position to start
    int ngroup = 0;
    if (ktime) {
        while ((int)ctx->kev.size() < 8) {
            hipEvent_t e = nullptr;
            HIPCHK(hipEventCreate(&e));
            ctx->kev.push_back(e);
        }
    }
    const int* pos = ctx->d_pos.as<int>();
    // one check group of iterations of a lane; a timed group counts the
    // active slots before its second iteration and launches the product and
    // update of its second and third iterations with events that take the
    // time stamps of their own dispatch packets (two consecutive iterations:
    // the update writes lambda in every other one)
    // the graph holds `gcap` iterations and is launched group / gcap times per
    // check group, so that the re-capture after a refill or compaction is short
    const int gcap = (group > 16 && group % 16 == 0) ? 16 : group;
    auto n_timed = [](int iters) { return iters > 2 ? 2 : 1; };
    auto body = [&](Lane& L, bool timed_group, int iters) -> hipError_t {
        const int tq = iters > 1 ? 1 : 0, nt = n_timed(iters);
        hipError_t e = hipSuccess;
        for (int q = 0; q < iters && e == hipSuccess; ++q) {
            const int ti = q - tq;
            const bool timed = timed_group && ti >= 0 && ti < nt;
            if (timed && ti == 0 && (e = launch_count_active(L.a.active, L.S, L.a.any_active + 1, L.s)) != hipSuccess)
                break;
            hipEvent_t* ev = timed ? &ctx->kev[4 * ti] : nullptr;
            e = launch_cg_apply_mfma(L.a, L.a.p, L.Y, ctx->SR, L.G->d_work.as<int4>(), L.G->nwork,
                                     L.G->d_perm.as<int>(), ctx->max_R, L.s, ev ? ev[0] : nullptr,
                                     ev ? ev[1] : nullptr);
            if (e == hipSuccess)
                e = launch_cg_update2(L.a, L.Y, ctx->SR, pos, L.s, ev ? ev[2] : nullptr, ev ? ev[3] : nullptr);
        }
        return e;
    };
    auto capture = [&](Lane& L) -> int {
        L.release();
        if (!ctx->opt_graph) return SDMM_OK;
        HIPCHK(hipStreamBeginCapture(L.s, hipStreamCaptureModeThreadLocal));
        hipError_t e = body(L, false, gcap);
        hipError_t e2 = hipStreamEndCapture(L.s, &L.graph);
        if (e != hipSuccess || e2 != hipSuccess) {
            if (L.graph) (void)hipGraphDestroy(L.graph);
            L.graph = nullptr;
            return fail(ctx, SDMM_EDEVICE, "graph capture of the CG iterations failed");
        }
        if (hipGraphInstantiate(&L.exec, L.graph, nullptr, nullptr, 0) != hipSuccess) {
            (void)hipGraphDestroy(L.graph);
            L.graph = nullptr;
            L.exec = nullptr;
            return fail(ctx, SDMM_EDEVICE, "graph instantiation failed");
        }
        return SDMM_OK;
    };
    // pending realizations into the lane's free slots, and their CG started
    auto admit = [&](Lane& L) -> int {
        L.init.clear();
        for (int64_t l = 0; l < L.S && next < n; ++l) {
            if (L.slot_q[l] >= 0) continue;
            L.slot_q[l] = (int)next;
            L.slot_g[l] = ctx->h_gidx[next];
            ++next;
            L.init.push_back((int)l);
        }
        if (L.init.empty()) return SDMM_OK;
        HIPCHK(hipMemcpyAsync(ctx->w_slot_q.as<int>() + L.base, L.slot_q.data(), L.S * 4, hipMemcpyHostToDevice,
                              L.s));
        HIPCHK(hipMemcpyAsync(ctx->w_init.as<int>() + L.base, L.init.data(), L.init.size() * 4,
                              hipMemcpyHostToDevice, L.s));
        HIPCHK(launch_cg_init(L.a, (int64_t)L.init.size(), L.s));
        HIPCHK(hipStreamSynchronize(L.s));   // the host vectors change before the next admission
        return SDMM_OK;
    };
    // finished realizations leave the lane's slots (all occupied slots when `all`)
    auto retire = [&](Lane& L, bool all) -> int {
        HIPCHK(hipMemcpyAsync(L.act.data(), L.a.active, L.S * 4, hipMemcpyDeviceToHost, L.s));
        HIPCHK(hipMemcpyAsync(L.itv.data(), L.a.iters, L.S * 4, hipMemcpyDeviceToHost, L.s));
        HIPCHK(hipMemcpyAsync(L.stv.data(), L.a.status, L.S * 4, hipMemcpyDeviceToHost, L.s));
        HIPCHK(hipStreamSynchronize(L.s));
        for (int64_t l = 0; l < L.S; ++l) {
            if (L.slot_q[l] < 0 || (L.act[l] && !all)) continue;
            tot_it += L.itv[l];
            bad |= L.stv[l] != SDMM_CG_CONVERGED;
            brk |= L.stv[l] == SDMM_CG_BREAKDOWN;
            L.slot_q[l] = -1;
        }
        return SDMM_OK;
    };
    // operator work over the lane's occupied slots, and a new graph for it
    auto regroup = [&](Lane& L) -> int {
        L.sel.clear();
        for (int64_t l = 0; l < L.S; ++l)
            if (L.slot_q[l] >= 0) L.sel.push_back((int)l);
        int r2;
        if ((r2 = build_groups(ctx, *L.G, L.S, &L.sel, L.slot_g.data(), L.s))) return r2;
        L.in_work = (int64_t)L.sel.size();
        return capture(L);
    };
    // queue the lane's next check group and the read-back of its active count
    auto launch = [&](Lane& L) -> int {
        L.timed = ktime && L.id == 0 && (ngroup++ % kTimeEvery == 0);
        hipError_t e = hipSuccess;
        // the timed iteration runs alone on the device: the other lane's
        // group is drained first and its next group waits for the timed pair
        Lane* other = (L.timed && nl == 2 && !lanes[1].done) ? &lanes[1] : nullptr;
        if (other) HIPCHK(hipStreamSynchronize(other->s));
        if (L.exec && !L.timed) {
            for (int j = 0; j < group / gcap && e == hipSuccess; ++j) e = hipGraphLaunch(L.exec, L.s);
        } else {
            e = body(L, L.timed, group);
        }
        if (e == hipSuccess && other) e = hipStreamWaitEvent(other->s, ctx->kev[3], 0);
        if (e == hipSuccess) e = launch_count_active(L.a.active, L.S, L.a.any_active, L.s);
        if (e == hipSuccess) e = hipMemcpyAsync(ctx->h_count + 2 * L.id, L.a.any_active, 8, hipMemcpyDeviceToHost, L.s);
        if (e != hipSuccess) return fail(ctx, SDMM_EDEVICE, hipGetErrorString(e));
        ctx->counters.cg_launches += group;
        ++L.groups;
        return SDMM_OK;
    };
    // the lane's group has finished: timing, then retire / refill / compact
    auto service = [&](Lane& L) -> int {
        HIPCHK(hipStreamSynchronize(L.s));
        const int32_t count = ctx->h_count[2 * L.id], tactive = ctx->h_count[2 * L.id + 1];
        if (L.timed) {
            // the active count of the first timed iteration stands for both
            const int nt = n_timed(group);
            for (int ti = 0; ti < nt; ++ti) {
                float ma = 0.f, mu = 0.f;
                HIPCHK(hipEventElapsedTime(&ma, ctx->kev[4 * ti], ctx->kev[4 * ti + 1]));
                HIPCHK(hipEventElapsedTime(&mu, ctx->kev[4 * ti + 2], ctx->kev[4 * ti + 3]));
                ctx->counters.ms_cg_apply += ma;
                ctx->counters.ms_cg_update += mu;
                ctx->counters.cg_timed_launches += 1;
                ctx->counters.cg_timed_active += tactive;
                ctx->counters.cg_timed_columns += L.in_work;
            }
        }
        int r2;
        const int64_t refill = std::max<int64_t>(1, L.S / 16);
        if (count == 0 && next >= n) {
            L.done = true;
            return retire(L, true);
        }
        if (next < n && L.S - count >= refill) {
            if ((r2 = retire(L, false)) || (r2 = admit(L)) || (r2 = regroup(L))) return r2;
        } else if (next >= n && count < 0.75 * L.in_work) {
            if ((r2 = retire(L, false)) || (r2 = regroup(L))) return r2;
        }
        return SDMM_OK;
    };
    auto release_all = [&]() {
        for (int k = 0; k < nl; ++k) lanes[k].release();
    };
    // the second lane starts after the work already queued on st
    if (nl == 2) {
        HIPCHK(hipEventRecord(ctx->lane_ev, st));
        HIPCHK(hipStreamWaitEvent(ctx->lane_stream, ctx->lane_ev, 0));
    }
    for (int k = 0; k < nl && !rc; ++k)
        if (!(rc = admit(lanes[k]))) rc = regroup(lanes[k]);
    // every realization stops within max_iter iterations of its start
    const int64_t max_groups = (n / std::max<int64_t>(1, S / (16 * nl)) + 2) * ((int64_t)max_iter / group + 2);
    for (int k = 0; k < nl && !rc; ++k) {
        Lane& L = lanes[k];
        if (L.in_work == 0) {
            L.done = true;
            continue;
        }
        rc = launch(L);
    }
    // round robin: each lane is serviced when its group ends and relaunched at
    // once, while the other lane's group keeps the device busy
    for (bool busy = true; busy && !rc;) {
        busy = false;
        for (int k = 0; k < nl && !rc; ++k) {
            Lane& L = lanes[k];
            if (L.done) continue;
            if (L.groups > max_groups) {
                rc = fail(ctx, SDMM_EDEVICE, "the CG driver did not finish");
                break;
            }
            if ((rc = service(L))) break;
            if (!L.done) {
                if ((rc = launch(L))) break;
                busy = true;
            }
        }
    }
    // nothing of either lane is in flight when their graphs are destroyed
    for (int k = 0; k < nl; ++k) (void)hipStreamSynchronize(lanes[k].s);
    release_all();
    return rc;
}

hipStream_t work_stream(Prob* ctx, hipStream_t user) {
    // graph capture needs a stream other than the legacy null stream
    if (!ctx->opt_graph) return user;
    if (!ctx->cap_stream && hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking) != hipSuccess)
        ctx->cap_stream = nullptr;
    return ctx->cap_stream ? ctx->cap_stream : user;
}

}  // namespace

// ---- Method S2 (Section 5.3): a deterministic basis for every realization ----

constexpr int kDetChunkUnits = 1024;   // units built per launch (their factor scratch is reused)

// The points of a batch on the host: collocation points of gidx (device) or
// the caller's off-grid points y (device, n x n_term).
int det_points(Prob* ctx, int64_t n, const int64_t* gidx, const double* y, hipStream_t st, std::vector<double>& out) {
    const Problem& P = ctx->P;
    const int nt = P.nterm;
    out.assign((size_t)n * nt, 0.0);
    if (gidx) {
        int rc;
        if ((rc = check_indices(ctx, gidx, n, st)) || (rc = fetch_gidx(ctx, gidx, n, st))) return rc;
        for (int64_t q = 0; q < n; ++q)
            for (int t = 0; t < nt; ++t) out[(size_t)q * nt + t] = P.node_x[P.ids[(size_t)ctx->h_gidx[q] * nt + t]];
    } else if (nt > 0) {
        HIPCHK(hipMemcpyAsync(out.data(), y, out.size() * 8, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        for (double v : out)
            if (!std::isfinite(v)) return fail(ctx, SDMM_EINVAL, "a point coordinate is not finite");
    }
    return SDMM_OK;
}

// Units, offsets, device tables and the basis view of a batch of n
// realizations.  resident: every unit keeps its own factor scratch (Method
// S1 solves with the factors in every CG iteration); otherwise the scratch
// is reused chunk by chunk.
int det_layout(Prob* ctx, int64_t n, hipStream_t st, bool resident = false) {
    Problem& P = ctx->P;
    DetBatch& D = ctx->det;
    BasisView& V = D.view;
    const int nsub = (int)P.subs.size(), nr = P.n_region;
    D.units.clear();
    D.chunk_start.clear();
    V.pair_sub.clear();
    V.pair_k.clear();
    std::vector<int64_t> sbase(nsub, 0), abase(nsub, 0), dabase;
    std::vector<int> unit_of_dk, dnl;
    int64_t S_off = 0, X_off = 0, A_off = ctx->A_total;
    for (int i = 0; i < nsub; ++i) {
        sbase[i] = S_off;
        const int R = ctx->sub_R[i];
        if (ctx->sub_region[i] >= 0) {
            S_off += n * (int64_t)R * R;
            abase[i] = A_off;
            A_off += n * ((int64_t)R + (int64_t)R * R);
        } else {
            S_off += (int64_t)R * R;
            abase[i] = ctx->sub_Abase[i];
        }
    }
    D.A_base = ctx->A_total;
    int64_t L_off = 0, T_off = 0, I_off = 0, L_max = 0, T_max = 0, I_max = 0;
    int in_chunk = 0;
    unit_of_dk.assign(P.darcy.size() * (size_t)n, -1);
    // order: the units built through the LDS window, chunk by chunk
    // (chunk_start indexes it); wide: the exact-mass units that go through
    // the tiled band LDL^T instead
    std::vector<int> order, wide;
    for (size_t di = 0; di < P.darcy.size(); ++di) {
        const DarcyHost& h = P.darcy[di];
        const int i = h.sub, r = P.subs[i].region;
        const int64_t Np = (h.Ns + 15) / 16 * 16, bp = (h.bs + 15) / 16 * 16;
        const bool is_wide = bp > kMaxDarcyBand;
        dabase.push_back(abase[i]);
        dnl.push_back((int)n);
        for (int64_t q = 0; q < n; ++q) {
            UnitDev u{};
            u.d = (int)di;
            u.k = (int)q;
            u.sub = i;
            u.off_xi = q * P.nterm + P.dim_off[r];
            u.off_S = sbase[i] + q * (int64_t)h.R * h.R;
            u.off_X = X_off;
            X_off += Np * h.R;
            if (is_wide) {
                wide.push_back((int)D.units.size());
            } else {
                if (in_chunk == 0) {
                    D.chunk_start.push_back((int)order.size());
                    L_off = T_off = I_off = 0;
                }
                u.off_L = L_off;
                u.off_T = T_off;
                u.off_I = I_off;
                L_off += Np * (bp + 1);
                T_off += darcy_tscr(h);
                I_off += Np * 16;
                L_max = std::max(L_max, L_off);
                T_max = std::max(T_max, T_off);
                I_max = std::max(I_max, I_off);
                order.push_back((int)D.units.size());
                if (++in_chunk == kDetChunkUnits && !resident) in_chunk = 0;
            }
            unit_of_dk[di * (size_t)n + q] = (int)D.units.size();
            D.units.push_back(u);
            V.pair_sub.push_back(i);
            V.pair_k.push_back((int)q);
        }
    }
    D.chunk_start.push_back((int)order.size());
    // the wide units keep K of their cells (the flux readout reads it) after
    // the window units' scratch
    for (int u : wide) {
        D.units[u].off_T = T_max;
        T_max += P.darcy[D.units[u].d].N;
    }
    for (size_t si = 0; si < P.stokes.size(); ++si) {
        V.pair_sub.push_back(P.stokes[si].sub);
        V.pair_k.push_back(0);
    }
    V.g2l.assign((size_t)n * nr, 0);
    for (int64_t q = 0; q < n; ++q)
        for (int r = 0; r < nr; ++r) V.g2l[(size_t)q * nr + r] = (int32_t)q;
    V.nlocal.assign(nr, (int)n);
    int rc;
    auto grow = [&](DevBuf& b, size_t bytes) { return b.bytes < bytes ? alloc(ctx, b, bytes) : SDMM_OK; };
    const bool mixed = D.precision == SDMM_PREC_MIXED;
    if ((rc = grow(D.d_S, S_off * 8)) || (rc = grow(D.d_X, X_off * 8)) || (rc = grow(D.d_T, T_max * 8)) ||
        (rc = grow(D.d_refine, 16)))
        return rc;
    if (mixed) {
        if ((rc = grow(D.d_E, X_off * 8)) || (rc = grow(D.d_W32, X_off * 4)) || (rc = grow(D.d_L32, L_max * 4)) ||
            (rc = grow(D.d_I32, std::max<int64_t>(I_max, 1) * 4)))
            return rc;
    } else if ((rc = grow(D.d_L, L_max * 8)) || (rc = grow(D.d_I, std::max<int64_t>(I_max, 1) * 8))) {
        return rc;
    }
    // accumulators: the stochastic layout, then the batch's Darcy pairs;
    // what the first part holds (the Stokes accumulators) is kept
    if (ctx->d_acc.bytes < (size_t)A_off * 8) {
        DevBuf nb;
        if ((rc = alloc(ctx, nb, A_off * 8))) return rc;
        HIPCHK(hipMemsetAsync(nb.p, 0, nb.bytes, st));
        HIPCHK(hipMemcpyAsync(nb.p, ctx->d_acc.p, ctx->d_acc.bytes, hipMemcpyDeviceToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
        std::swap(ctx->d_acc.p, nb.p);
        std::swap(ctx->d_acc.bytes, nb.bytes);
        std::swap(ctx->d_acc.al, nb.al);
    }
    std::vector<StokesDev> wsdx;
    plan_wide(P, D.units, wide, ctx->wt_cap_tiles, ctx->wt_cap_rhs, ctx->wt_cap_linv, D.wide_chunks, wsdx);
    if (!wide.empty() && ((rc = upload_on(ctx, D.d_wide_sdx, wsdx, st)) || (rc = upload_on(ctx, D.d_wide_units, wide, st))))
        return rc;
    // every unit wide: no window chunk reads the order list, but its buffer
    // is still uploaded
    if (order.empty()) order.push_back(0);
    std::vector<int64_t> pos(n);
    for (int64_t q = 0; q < n; ++q) pos[q] = q;
    if ((rc = upload_on(ctx, D.d_units, D.units, st)) || (rc = upload_on(ctx, D.d_order, order, st)) ||
        (rc = upload_on(ctx, D.d_pos, pos, st)) || (rc = upload_on(ctx, D.d_unit_of_dk, unit_of_dk, st)) ||
        (rc = upload_on(ctx, D.d_dnlocal, dnl, st)) || (rc = upload_on(ctx, D.d_dAbase, dabase, st)) ||
        (rc = upload_on(ctx, V.d_pair_sub, V.pair_sub, st)) || (rc = upload_on(ctx, V.d_pair_k, V.pair_k, st)) ||
        (rc = upload_on(ctx, V.d_sub_Sbase, sbase, st)) || (rc = upload_on(ctx, V.d_sub_Abase, abase, st)))
        return rc;
    const int64_t nd = 2 * (ctx->field_size[1] + ctx->field_size[2]);
    if ((rc = grow(D.d_tmp, std::max<int64_t>(nd, 1) * 8))) return rc;
    if (!D.d_sum.p) {
        if ((rc = alloc(ctx, D.d_sum, std::max<int64_t>(nd, 1) * 8))) return rc;
        HIPCHK(hipMemsetAsync(D.d_sum.p, 0, D.d_sum.bytes, st));
        HIPCHK(hipStreamSynchronize(st));
    }
    V.S = D.d_S.as<double>();
    D.S_total = S_off;
    D.X_total = X_off;
    D.n = n;
    return SDMM_OK;
}

// Build the deterministic bases of the batch (Section 5.3: S_{H,i} of every
// Darcy subdomain from the realization's own KL field, eqs. starDproblem1-2);
// the Stokes blocks, which no realization changes, are copied from the
// Stokes build.
int det_build(Prob* ctx, const std::vector<double>& y, hipStream_t st) {
    DetBatch& D = ctx->det;
    int rc;
    if (!y.empty()) {
        if ((rc = upload_on(ctx, D.d_xi, y, st))) return rc;
    } else if ((rc = alloc(ctx, D.d_xi, 8))) {
        return rc;
    }
    DarcyTables t = darcy_tables(ctx);
    t.units = D.d_units.as<UnitDev>();
    t.order = D.d_order.as<int>();
    t.xi = D.d_xi.as<double>();
    int max_np = 0;   // over the units of the LDS window
    for (auto& h : ctx->P.darcy)
        if ((h.bs + 15) / 16 * 16 <= kMaxDarcyBand) max_np = std::max(max_np, (h.Ns + 15) / 16 * 16);
    const bool mixed = D.precision == SDMM_PREC_MIXED;
    if (mixed) HIPCHK(hipMemsetAsync(D.d_refine.p, 0, 16, st));
    if (!D.wide_chunks.empty() &&
        (rc = darcy_build_wide(ctx, t, D.wide_chunks, D.d_wide_sdx, D.d_wide_units, D.d_X.as<double>(),
                               D.d_S.as<double>(), D.d_T.as<double>(), st)))
        return rc;
    for (size_t c = 0; c + 1 < D.chunk_start.size(); ++c) {
        t.unit_base = D.chunk_start[c];
        const int count = D.chunk_start[c + 1] - D.chunk_start[c];
        if (count <= 0) continue;
        if (mixed)
            HIPCHK(launch_darcy_basis_blocked_mixed(t, count, ctx->max_b, ctx->max_Rd, max_np, 0, D.d_S.as<double>(),
                                                    D.d_X.as<double>(), D.d_E.as<double>(), D.d_L32.as<float>(),
                                                    D.d_I32.as<float>(), D.d_T.as<double>(), D.d_W32.as<float>(),
                                                    kMaxRefine, kRefineTol, D.d_refine.as<double>(),
                                                    reinterpret_cast<int*>(D.d_refine.as<char>() + 8), st));
        else
            HIPCHK(launch_darcy_basis_blocked(t, count, ctx->max_b, ctx->max_Rd, max_np, 0, D.d_S.as<double>(),
                                              D.d_X.as<double>(), D.d_L.as<double>(), D.d_I.as<double>(),
                                              D.d_T.as<double>(), ctx->P.in.darcy_mass, st));
    }
    const Problem& P = ctx->P;
    std::vector<int64_t> sbase(P.subs.size());
    HIPCHK(hipMemcpyAsync(sbase.data(), D.view.d_sub_Sbase.p, sbase.size() * 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (auto& sh : P.stokes) {
        const int i = sh.sub, R = ctx->sub_R[i];
        HIPCHK(hipMemcpyAsync(D.d_S.as<double>() + sbase[i], ctx->d_S.as<double>() + ctx->sub_Sbase[i],
                              (size_t)R * R * 8, hipMemcpyDeviceToDevice, st));
    }
    if (mixed) {
        double mr = 0.0;
        HIPCHK(hipMemcpyAsync(&mr, D.d_refine.p, 8, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        ctx->counters.max_refine_residual = mr;
        if (!(mr <= kRefineTol))
            return fail(ctx, SDMM_ENOTCONV, "mixed-precision refinement of a deterministic basis stopped at " +
                                                std::to_string(mr));
    }
    int64_t sd = 0;
    for (auto& u : D.units) sd += ctx->P.darcy[u.d].R;
    ctx->counters.basis_solves_darcy += sd;
    ctx->counters.units_built += (int64_t)D.units.size();
    return SDMM_OK;
}

// ---- Method S1 (Section 5.2) ------------------------------------------------

int accumulate_core(Prob* ctx, int64_t n, const int64_t* grp_idx, const int64_t* w_idx, const double* lambda,
                    const double* weights, hipStream_t st, int64_t chunk_override = 0, bool alpha_ready = false);

// Factors of every (Darcy subdomain, realization) unit of the batch (each
// realization's own KL field, eqs. KLapprox and starDproblem1-2), kept
// resident for the local solves of every CG iteration, the local-solution
// scratch, and the work list of the Stokes products (their responses do not
// depend on the realization, R2).
int s1_prepare(Prob* ctx, int64_t n, const std::vector<double>& pts, hipStream_t st) {
    DetBatch& D = ctx->det;
    const Problem& P = ctx->P;
    int rc;
    for (auto& h : P.darcy)
        if (h.R > kS1MaxR || h.n_medge > kS1MaxMedge)
            return fail(ctx, SDMM_EINVAL, "Method S1 handles at most 256 mortar DOFs and 512 mortar edges per Darcy subdomain");
    D.precision = SDMM_PREC_FP64;
    if ((rc = det_layout(ctx, n, st, true))) return rc;
    if (!pts.empty()) {
        if ((rc = upload(ctx, D.d_xi, pts))) return rc;
    } else if ((rc = alloc(ctx, D.d_xi, 8))) {
        return rc;
    }
    int max_np = 0;
    for (auto& h : P.darcy) max_np = std::max(max_np, (h.N + 15) / 16 * 16);
    const int64_t zn = n * (int64_t)P.darcy.size() * max_np;
    if (D.d_z.bytes < (size_t)std::max<int64_t>(zn, 1) * 8 && (rc = alloc(ctx, D.d_z, std::max<int64_t>(zn, 1) * 8)))
        return rc;
    DarcyTables t = darcy_tables(ctx);
    t.units = D.d_units.as<UnitDev>();
    t.order = D.d_order.as<int>();
    t.xi = D.d_xi.as<double>();
    t.unit_base = 0;
    HIPCHK(launch_darcy_factor_only(t, (int)D.units.size(), ctx->max_b, max_np, D.d_X.as<double>(),
                                    D.d_L.as<double>(), D.d_I.as<double>(), D.d_T.as<double>(), st));
    std::vector<int4> work;
    for (auto& sh : P.stokes) {
        const int i = sh.sub, R = ctx->sub_R[i];
        for (int64_t c0 = 0; c0 < n; c0 += 64) {
            const int cnt = (int)std::min<int64_t>(64, n - c0);
            for (int row0 = 0; row0 < R; row0 += 64) work.push_back(make_int4(i, 0, row0 | (cnt << 16), (int)c0));
        }
    }
    std::vector<int> perm(n);
    for (int64_t q = 0; q < n; ++q) perm[q] = (int)q;
    D.s1_nwork = (int)work.size();
    if (work.empty()) work.push_back(make_int4(0, 0, 0, 0));
    if ((rc = upload(ctx, D.d_s1work, work)) || (rc = upload(ctx, D.d_s1perm, perm))) return rc;
    return SDMM_OK;
}

// S_H x for the n vectors of x (global layout) into Y (subdomain-local
// layout): local Darcy solves with the batch's factors and the Stokes
// responses; vectors with active == 0 are skipped on the Darcy side.
hipError_t s1_apply(Prob* ctx, const CgArgs& a, int64_t n, const int32_t* active, const double* x, double* Y,
                    hipStream_t st) {
    DetBatch& D = ctx->det;
    const Problem& P = ctx->P;
    DarcyTables t = darcy_tables(ctx);
    t.units = D.d_units.as<UnitDev>();
    t.order = D.d_order.as<int>();
    t.xi = D.d_xi.as<double>();
    int max_np = 0;
    for (auto& h : P.darcy) max_np = std::max(max_np, (h.N + 15) / 16 * 16);
    hipError_t e = launch_darcy_s1_apply(t, D.d_unit_of_dk.as<int>(), (int)n, (int)n, nullptr, active, x, P.M,
                                         ctx->d_sub_dof_ptr.as<int64_t>(), ctx->d_sub_dofs.as<int64_t>(),
                                         D.d_L.as<double>(), D.d_I.as<double>(), D.d_T.as<double>(),
                                         D.d_X.as<double>(), D.d_z.as<double>(), (int)P.darcy.size(), max_np,
                                         ctx->max_b, Y, ctx->SR, st);
    if (e != hipSuccess) return e;
    return launch_cg_apply_mfma(a, x, Y, ctx->SR, D.d_s1work.as<int4>(), D.s1_nwork, D.d_s1perm.as<int>(),
                                ctx->max_R, st);
}

// Method S1: CG for the whole batch at once (every realization holds a slot
// until it stops), S_H applied through local solves in every iteration.
int s1_solve(Prob* ctx, int64_t n, const int64_t* gidx, const double* y, double rtol, int32_t max_iter,
             double* lambda, int32_t* iters, double* relres, int32_t* status, hipStream_t st) {
    DetBatch& D = ctx->det;
    const Problem& P = ctx->P;
    int rc;
    std::vector<double> pts;
    D.valid = false;
    if ((rc = det_points(ctx, n, gidx, y, st, pts)) || (rc = s1_prepare(ctx, n, pts, st))) return rc;
    if ((rc = ensure_workspace(ctx, n))) return rc;
    CgArgs a = cg_args(ctx, n, D.d_pos.as<int64_t>(), lambda);
    std::vector<int> ident(n);
    for (int64_t q = 0; q < n; ++q) ident[q] = (int)q;
    HIPCHK(hipMemcpyAsync(ctx->w_slot_q.p, ident.data(), n * 4, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(ctx->w_init.p, ident.data(), n * 4, hipMemcpyHostToDevice, st));
    a.slot_q = ctx->w_slot_q.as<int>();
    a.init_slots = ctx->w_init.as<int>();
    a.rtol = rtol;
    a.max_iter = max_iter;
    a.iters_out = iters;
    a.relres_out = relres;
    a.status_out = status;
    HIPCHK(hipEventRecord(ctx->ev[3], st));
    HIPCHK(launch_cg_init(a, n, st));
    double* Y = ctx->w_Y.as<double>();
    const int* pos = ctx->d_pos.as<int>();
    const int group = ctx->opt_check;
    const int64_t max_groups = (int64_t)max_iter / group + 2;
    for (int64_t grp = 0;; ++grp) {
        if (grp > max_groups) return fail(ctx, SDMM_EDEVICE, "the CG driver did not finish");
        for (int q = 0; q < group; ++q) {
            HIPCHK(s1_apply(ctx, a, n, a.active, a.p, Y, st));
            HIPCHK(launch_cg_update2(a, Y, ctx->SR, pos, st));
        }
        HIPCHK(launch_count_active(a.active, n, a.any_active, st));
        int32_t count = 0;
        HIPCHK(hipMemcpyAsync(&count, a.any_active, 4, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (count == 0) break;
    }
    HIPCHK(hipEventRecord(ctx->ev[4], st));
    std::vector<int32_t> itv(2 * n);
    HIPCHK(hipMemcpyAsync(itv.data(), a.iters, n * 4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(itv.data() + n, a.status, n * 4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    int64_t tot = 0;
    bool bad = false, brk = false;
    for (int64_t l = 0; l < n; ++l) {
        tot += itv[l];
        bad |= itv[n + l] != SDMM_CG_CONVERGED;
        brk |= itv[n + l] == SDMM_CG_BREAKDOWN;
    }
    ctx->counters.cg_iterations += tot;
    ctx->counters.realizations += n;
    // one local solve per Darcy subdomain in every iteration (eq. S1-cost)
    ctx->counters.basis_solves_darcy += tot * (int64_t)P.darcy.size();
    ctx->counters.units_built += (int64_t)D.units.size();
    float ms = 0;
    if (hipEventElapsedTime(&ms, ctx->ev[3], ctx->ev[4]) == hipSuccess) ctx->counters.ms_solve = ms;
    D.y = pts;
    D.valid = true;
    if (brk) return fail(ctx, SDMM_EBREAKDOWN, "CG breakdown in some realization");
    if (bad) return fail(ctx, SDMM_ENOTCONV, "some realization reached max_iter");
    return SDMM_OK;
}

// Method S1 moments: lambda and the Stokes fields through the reduced form
// (as for every method), the Darcy fields of each realization from one
// recovery solve per subdomain with its final lambda, summed with the
// weights into the batch sums.
int s1_accumulate(Prob* ctx, int64_t n, const int64_t* gidx, const double* lambda, const double* weights,
                  hipStream_t st) {
    DetBatch& D = ctx->det;
    const Problem& P = ctx->P;
    int rc;
    if ((rc = ensure_workspace(ctx, n))) return rc;
    CgArgs a = cg_args(ctx, n, D.d_pos.as<int64_t>(), const_cast<double*>(lambda));
    // S_H lambda (its Darcy solves leave z = P^{-1} E lambda_i in the scratch)
    HIPCHK(s1_apply(ctx, a, n, nullptr, lambda, ctx->w_Y.as<double>(), st));
    if (P.n_kernel > 0) {
        HIPCHK(launch_gather_global(ctx->w_Y.as<double>(), ctx->SR, ctx->d_pos.as<int>(), P.M, n,
                                    ctx->w_Slam.as<double>(), st));
        HIPCHK(launch_alpha(a, ctx->w_Slam.as<double>(), ctx->w_alpha.as<double>(), st));
    }
    int64_t a_n = 0;
    for (auto& h : P.darcy) a_n += n * ((int64_t)h.R + (int64_t)h.R * h.R);
    HIPCHK(hipMemsetAsync(ctx->d_acc.as<double>() + D.A_base, 0, a_n * 8, st));
    ctx->view = &D.view;
    rc = accumulate_core(ctx, n, D.d_pos.as<int64_t>(), gidx, lambda, weights, st, n, true);
    ctx->view = nullptr;
    if (rc) return rc;
    const int64_t f1 = ctx->field_size[1], f2 = ctx->field_size[2];
    if (D.d_F.bytes < (size_t)std::max<int64_t>(n * (f1 + f2), 1) * 8 &&
        (rc = alloc(ctx, D.d_F, std::max<int64_t>(n * (f1 + f2), 1) * 8)))
        return rc;
    DarcyTables t = darcy_tables(ctx);
    t.units = D.d_units.as<UnitDev>();
    t.order = D.d_order.as<int>();
    t.xi = D.d_xi.as<double>();
    int max_np = 0;
    for (auto& h : P.darcy) max_np = std::max(max_np, (h.N + 15) / 16 * 16);
    HIPCHK(launch_darcy_s1_moments(t, D.d_unit_of_dk.as<int>(), (int)n, lambda, P.M, ctx->d_sub_dof_ptr.as<int64_t>(),
                                   ctx->d_sub_dofs.as<int64_t>(), D.d_z.as<double>(), (int)P.darcy.size(), max_np,
                                   ctx->d_cell_out.as<int64_t>(), ctx->d_edge_out.as<int64_t>(), f1, f2,
                                   D.d_F.as<double>(), weights, gidx, ctx->d_weights.as<double>(),
                                   D.d_sum.as<double>(), st));
    HIPCHK(hipStreamSynchronize(st));
    ctx->counters.basis_solves_darcy += n * (int64_t)P.darcy.size();   // the recovery solves
    ctx->moments_final = false;
    return SDMM_OK;
}

int impl_solve_interface(Prob* ctx, int64_t n, const int64_t* gidx, const double* y, double rtol, int32_t max_iter,
                         double* lambda, int32_t* iters, double* relres, int32_t* status, void* stream) {
    if (!ctx) return SDMM_EINVAL;
    ctx->view = nullptr;
    const bool det = ctx->method == SDMM_METHOD_DETERMINISTIC;
    const bool s1 = ctx->method == SDMM_METHOD_PER_ITERATION;
    const bool offgrid_ok = det || s1;
    if (n > 0 && !gidx && y && !offgrid_ok)
        return fail(ctx, SDMM_EINVAL, "off-grid points need Method S2 or S1 (a stochastic basis exists only on the grid)");
    if (ctx->host_only) return fail(ctx, SDMM_ESTATE, "context has no device");
    if (!ctx->basis_built) return fail(ctx, SDMM_ESTATE, "basis not built");
    if (n < 0 || (n > 0 && ((!gidx && !(offgrid_ok && y)) || !lambda)) || !(rtol > 0) || max_iter < 1)
        return fail(ctx, SDMM_EINVAL, "invalid arguments");
    if (n == 0) return SDMM_OK;
    if (n > 2147483647LL) return fail(ctx, SDMM_EINVAL, "batch too large");
    HIPCHK(hipSetDevice(ctx->device));
    hipStream_t user = (hipStream_t)stream;
    hipStream_t st = work_stream(ctx, user);
    HIPCHK(hipEventRecord(ctx->ev[5], user));
    HIPCHK(hipStreamWaitEvent(st, ctx->ev[5], 0));
    int rc;
    if (s1) {
        rc = s1_solve(ctx, n, gidx, y, rtol, max_iter, lambda, iters, relres, status, st);
        HIPCHK(hipEventRecord(ctx->ev[4], st));
        HIPCHK(hipStreamWaitEvent(user, ctx->ev[4], 0));
        return rc;
    }
    const int64_t* cg_idx = gidx;
    if (det) {
        // Method S2: this batch's own bases, then the CG on them (the batch
        // positions stand in for the global indices)
        std::vector<double> pts;
        ctx->det.valid = false;
        if ((rc = det_points(ctx, n, gidx, y, st, pts)) || (rc = det_layout(ctx, n, st))) return rc;
        rc = det_build(ctx, pts, st);
        if (rc && rc != SDMM_ENOTCONV) return rc;
        ctx->det.y = pts;
        ctx->det.valid = true;
        cg_idx = ctx->det.d_pos.as<int64_t>();
        ctx->view = &ctx->det.view;
    } else if ((rc = check_indices(ctx, gidx, n, st))) {
        return rc;
    }
    const int64_t chunk = chunk_size(ctx, n);
    if ((rc = ensure_workspace(ctx, chunk))) {
        ctx->view = nullptr;
        return rc;
    }
    HIPCHK(hipEventRecord(ctx->ev[3], st));
    int64_t tot = 0;
    bool bad = false, brk = false;
    rc = solve_batch(ctx, n, chunk, cg_idx, rtol, max_iter, lambda, iters, relres, status, st, tot, bad, brk);
    ctx->view = nullptr;
    if (rc) return rc;
    HIPCHK(hipEventRecord(ctx->ev[4], st));
    HIPCHK(hipStreamWaitEvent(user, ctx->ev[4], 0));
    HIPCHK(hipStreamSynchronize(st));
    ctx->counters.cg_iterations += tot;
    ctx->counters.realizations += n;
    float ms = 0;
    if (hipEventElapsedTime(&ms, ctx->ev[3], ctx->ev[4]) == hipSuccess) ctx->counters.ms_solve = ms;
    if (brk) return fail(ctx, SDMM_EBREAKDOWN, "CG breakdown in some realization");
    if (bad) return fail(ctx, SDMM_ENOTCONV, "some realization reached max_iter");
    return SDMM_OK;
}

// The CG of sdmm_solve_interface without any allocation: every realization
// of the batch holds one CG slot for the whole solve, the slot state and the
// group tables live in the device's fixed scratch array, the iterations are
// launched eagerly on the caller's stream (no graph, no second lane, no
// timing events), and the host reads the active count with a plain
// synchronous copy.  The kernels are those of the allocating path, so the
// results are the same.
int impl_solve_interface_noalloc(Prob* ctx, int64_t n, const int64_t* gidx, double rtol, int32_t max_iter,
                                 double* lambda, int32_t* iters, double* relres, int32_t* status, void* stream) {
    if (!ctx) return SDMM_EINVAL;
    if (ctx->method != SDMM_METHOD_STOCHASTIC)
        return fail(ctx, SDMM_ESTATE, "needs a stochastic basis (Method S3); this problem was built for Method S1 or S2");
    if (ctx->host_only) return fail(ctx, SDMM_ESTATE, "context has no device");
    if (!ctx->basis_built) return fail(ctx, SDMM_ESTATE, "basis not built");
    if (n < 0 || (n > 0 && (!gidx || !lambda)) || !(rtol > 0) || max_iter < 1)
        return fail(ctx, SDMM_EINVAL, "invalid arguments");
    if (n == 0) return SDMM_OK;
    if (n > 2147483647LL) return fail(ctx, SDMM_EINVAL, "batch too large");
    char* base = reinterpret_cast<char*>(noalloc_scratch_ptr(ctx->device));
    if (!base) return fail(ctx, SDMM_ESTATE, "the scratch array of this device was not resolved");
    HIPCHK(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    const Problem& P = ctx->P;
    const int M = P.M;
    // the indices, checked on the host before any kernel reads the table
    ctx->h_gidx.resize(n);
    HIPCHK(hipMemcpyAsync(ctx->h_gidx.data(), gidx, n * 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int64_t l = 0; l < n; ++l)
        if (ctx->h_gidx[l] < 0 || ctx->h_gidx[l] >= P.nreal)
            return fail(ctx, SDMM_EINVAL, "a global collocation index is out of range");
    Groups& G = ctx->grp_noalloc;
    int rc;
    if ((rc = build_groups_host(ctx, G, n, nullptr, ctx->h_gidx.data()))) return rc;
    // scratch layout (256-byte aligned pieces); the group tables get room for
    // the first grouping, which no later compaction exceeds
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) & ~(size_t)255;
        return o;
    };
    const size_t o_r = take((size_t)n * M * 8), o_p = take((size_t)n * M * 8), o_Y = take((size_t)n * ctx->SR * 8);
    const size_t o_rr = take(n * 8), o_r0 = take(n * 8), o_rel = take(n * 8), o_pend = take(n * 8);
    const size_t o_it = take(n * 4), o_stat = take(n * 4), o_act = take(n * 4), o_slot = take(n * 4),
                 o_init = take(n * 4), o_any = take(16);
    const size_t o_perm = take(G.h_perm.size() * 4), o_work = take(G.h_work.size() * 16);
    if (off > kNoAllocScratchBytes)
        return fail(ctx, SDMM_EINVAL,
                    "a batch of " + std::to_string(n) + " realizations needs " + std::to_string(off) +
                        " bytes of CG workspace, above the fixed " + std::to_string(kNoAllocScratchBytes) +
                        "-byte scratch of the allocation-free entry point");
    CgArgs a = cg_args(ctx, n, gidx, lambda);
    a.r = reinterpret_cast<double*>(base + o_r);
    a.p = reinterpret_cast<double*>(base + o_p);
    a.rr = reinterpret_cast<double*>(base + o_rr);
    a.r0 = reinterpret_cast<double*>(base + o_r0);
    a.pend = reinterpret_cast<double*>(base + o_pend);
    a.relres = reinterpret_cast<double*>(base + o_rel);
    a.iters = reinterpret_cast<int32_t*>(base + o_it);
    a.status = reinterpret_cast<int32_t*>(base + o_stat);
    a.active = reinterpret_cast<int32_t*>(base + o_act);
    a.any_active = reinterpret_cast<int32_t*>(base + o_any);
    int* d_slot = reinterpret_cast<int*>(base + o_slot);
    int* d_init = reinterpret_cast<int*>(base + o_init);
    a.slot_q = d_slot;
    a.init_slots = d_init;
    a.rtol = rtol;
    a.max_iter = max_iter;
    a.iters_out = iters;
    a.relres_out = relres;
    a.status_out = status;
    double* Y = reinterpret_cast<double*>(base + o_Y);
    int* d_perm = reinterpret_cast<int*>(base + o_perm);
    int4* d_work = reinterpret_cast<int4*>(base + o_work);
    auto upload_tables = [&]() -> int {
        HIPCHK(hipMemcpyAsync(d_perm, G.h_perm.data(), G.h_perm.size() * 4, hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(d_work, G.h_work.data(), G.h_work.size() * 16, hipMemcpyHostToDevice, st));
        HIPCHK(hipStreamSynchronize(st));   // the host tables change at the next compaction
        return SDMM_OK;
    };
    // slot l holds batch position l for the whole solve; cg_init sets every
    // slot's state, so nothing left in the scratch by an earlier call is read
    std::vector<int>& ident = ctx->noalloc_ident;
    ident.resize(n);
    for (int64_t l = 0; l < n; ++l) ident[l] = (int)l;
    HIPCHK(hipMemcpyAsync(d_slot, ident.data(), n * 4, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(d_init, ident.data(), n * 4, hipMemcpyHostToDevice, st));
    if ((rc = upload_tables())) return rc;
    HIPCHK(launch_cg_init(a, n, st));
    const int group = ctx->opt_check;
    const int* pos = ctx->d_pos.as<int>();
    int64_t in_work = n;
    const int64_t max_groups = (int64_t)max_iter / group + 2;
    std::vector<int32_t>& act = ctx->noalloc_act;
    for (int64_t grp = 0;; ++grp) {
        if (grp > max_groups) return fail(ctx, SDMM_EDEVICE, "the CG driver did not finish");
        for (int q = 0; q < group; ++q) {
            HIPCHK(launch_cg_apply_mfma(a, a.p, Y, ctx->SR, d_work, G.nwork, d_perm, ctx->max_R, st));
            HIPCHK(launch_cg_update2(a, Y, ctx->SR, pos, st));
        }
        HIPCHK(launch_count_active(a.active, n, a.any_active, st));
        int32_t count = 0;
        HIPCHK(hipMemcpyAsync(&count, a.any_active, 4, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (count == 0) break;
        if (count < 0.75 * in_work) {
            // compaction: the operator covers only the realizations still iterating
            act.resize(n);
            HIPCHK(hipMemcpyAsync(act.data(), a.active, n * 4, hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            std::vector<int>& sel = ctx->noalloc_sel;
            sel.clear();
            for (int64_t l = 0; l < n; ++l)
                if (act[l]) sel.push_back((int)l);
            if ((rc = build_groups_host(ctx, G, n, &sel, ctx->h_gidx.data()))) return rc;
            if ((rc = upload_tables())) return rc;
            in_work = (int64_t)sel.size();
        }
    }
    // per-realization status and the iteration total
    std::vector<int32_t>& itv = ctx->noalloc_act;
    itv.resize(2 * n);
    HIPCHK(hipMemcpyAsync(itv.data(), a.iters, n * 4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(itv.data() + n, a.status, n * 4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    int64_t tot = 0;
    bool bad = false, brk = false;
    for (int64_t l = 0; l < n; ++l) {
        tot += itv[l];
        bad |= itv[n + l] != SDMM_CG_CONVERGED;
        brk |= itv[n + l] == SDMM_CG_BREAKDOWN;
    }
    ctx->counters.cg_iterations += tot;
    ctx->counters.realizations += n;
    if (brk) return fail(ctx, SDMM_EBREAKDOWN, "CG breakdown in some realization");
    if (bad) return fail(ctx, SDMM_ENOTCONV, "some realization reached max_iter");
    return SDMM_OK;
}

// ---- CG streams (continuous batching of Section 5.4's main loop) -------------

int impl_stream_open(Prob* ctx, int64_t slots, double rtol, int32_t max_iter, void* stream, int64_t* sid) {
    if (!ctx || !sid) return SDMM_EINVAL;
    if (ctx->method != SDMM_METHOD_STOCHASTIC)
        return fail(ctx, SDMM_ESTATE, "needs a stochastic basis (Method S3); this problem was built for Method S1 or S2");
    if (ctx->host_only) return fail(ctx, SDMM_ESTATE, "context has no device");
    if (!ctx->basis_built) return fail(ctx, SDMM_ESTATE, "basis not built");
    if (slots < 1 || slots > (1 << 24) || !(rtol > 0) || max_iter < 1)
        return fail(ctx, SDMM_EINVAL, "invalid stream arguments");
    HIPCHK(hipSetDevice(ctx->device));
    std::unique_ptr<CgStream> cs(new (std::nothrow) CgStream());
    if (!cs) return fail(ctx, SDMM_ENOMEM, "stream");
    CgStream& c = *cs;
    c.S = slots;
    c.rtol = rtol;
    c.max_iter = max_iter;
    c.st = (hipStream_t)stream;
    const size_t S = slots, M = ctx->P.M;
    int rc;
    if ((rc = alloc(ctx, c.r, S * M * 8)) || (rc = alloc(ctx, c.p, S * M * 8)) ||
        (rc = alloc(ctx, c.Y, S * ctx->SR * 8)) || (rc = alloc(ctx, c.lam, S * M * 8)) ||
        (rc = alloc(ctx, c.rr, S * 8)) || (rc = alloc(ctx, c.r0, S * 8)) || (rc = alloc(ctx, c.pend, S * 8)) ||
        (rc = alloc(ctx, c.relres, S * 8)) ||
        (rc = alloc(ctx, c.iters, S * 4)) || (rc = alloc(ctx, c.status, S * 4)) ||
        (rc = alloc(ctx, c.active, S * 4)) || (rc = alloc(ctx, c.any, 16)) || (rc = alloc(ctx, c.slot_q, S * 4)) ||
        (rc = alloc(ctx, c.init, S * 4)) || (rc = alloc(ctx, c.g_slot, S * 4)) || (rc = alloc(ctx, c.g_lam, S * 8)) ||
        (rc = alloc(ctx, c.g_it, S * 8)) || (rc = alloc(ctx, c.g_rel, S * 8)) || (rc = alloc(ctx, c.g_st, S * 8)))
        return rc;
    // slot l holds its realization's state and outputs at row l
    std::vector<int> ident(S);
    for (size_t l = 0; l < S; ++l) ident[l] = (int)l;
    HIPCHK(hipMemcpy(c.slot_q.p, ident.data(), S * 4, hipMemcpyHostToDevice));
    HIPCHK(hipMemset(c.active.p, 0, S * 4));
    c.slot_g.assign(S, 0);
    c.slot_ticket.assign(S, -1);
    c.slot_row.assign(S, -1);
    c.act.assign(S, 0);
    *sid = ctx->next_stream++;
    ctx->streams[*sid] = std::move(cs);
    return SDMM_OK;
}

int find_stream(Prob* ctx, int64_t sid, CgStream** out) {
    auto it = ctx->streams.find(sid);
    if (it == ctx->streams.end()) return fail(ctx, SDMM_EINVAL, "unknown CG stream " + std::to_string(sid));
    *out = it->second.get();
    return SDMM_OK;
}

int impl_stream_submit(Prob* ctx, int64_t sid, int64_t n, const int64_t* gidx, double* lambda, int32_t* iters,
                       double* relres, int32_t* status, int64_t* ticket) {
    if (!ctx || !ticket) return SDMM_EINVAL;
    CgStream* c;
    int rc;
    if ((rc = find_stream(ctx, sid, &c))) return rc;
    if (n < 1 || n > 2147483647LL || !gidx || !lambda) return fail(ctx, SDMM_EINVAL, "invalid request");
    for (int64_t q = 0; q < n; ++q)
        if (gidx[q] < 0 || gidx[q] >= ctx->P.nreal)
            return fail(ctx, SDMM_EINVAL, "a global collocation index is out of range");
    const int64_t t = c->next_ticket++;
    c->reqs[t] = CgStream::Req{lambda, iters, relres, status, n};
    for (int64_t q = 0; q < n; ++q) c->queue.push_back({t, gidx[q], (int)q});
    *ticket = t;
    return SDMM_OK;
}

int impl_stream_run(Prob* ctx, int64_t sid, int32_t max_groups, int64_t* done, int64_t cap, int64_t* n_done,
                    int64_t* in_flight) {
    if (!ctx || !n_done || (cap > 0 && !done)) return SDMM_EINVAL;
    CgStream* cp;
    int rc;
    if ((rc = find_stream(ctx, sid, &cp))) return rc;
    CgStream& c = *cp;
    HIPCHK(hipSetDevice(ctx->device));
    *n_done = 0;
    const int M = ctx->P.M;
    CgArgs a = cg_args(ctx, c.S, nullptr, c.lam.as<double>());
    a.r = c.r.as<double>();
    a.p = c.p.as<double>();
    a.rr = c.rr.as<double>();
    a.r0 = c.r0.as<double>();
    a.pend = c.pend.as<double>();
    a.relres = c.relres.as<double>();
    a.iters = c.iters.as<int32_t>();
    a.status = c.status.as<int32_t>();
    a.active = c.active.as<int32_t>();
    a.any_active = c.any.as<int32_t>();
    a.slot_q = c.slot_q.as<int>();
    a.init_slots = c.init.as<int>();
    a.rtol = c.rtol;
    a.max_iter = c.max_iter;
    a.iters_out = nullptr;
    a.relres_out = nullptr;
    a.status_out = nullptr;
    const int* pos = ctx->d_pos.as<int>();
    std::vector<int64_t> finished;
    auto regroup = [&]() -> int {
        c.sel.clear();
        for (int64_t l = 0; l < c.S; ++l)
            if (c.slot_ticket[l] >= 0) c.sel.push_back((int)l);
        int r2;
        if ((r2 = build_groups_host(ctx, c.G, c.S, &c.sel, c.slot_g.data()))) return r2;
        if ((r2 = upload_groups(ctx, c.G, c.st))) return r2;
        c.in_work = (int64_t)c.sel.size();
        return SDMM_OK;
    };
    for (int32_t grp = 0; grp < std::max(1, max_groups); ++grp) {
        // admission: queued realizations into the free slots
        c.init_h.clear();
        for (int64_t l = 0; l < c.S && !c.queue.empty(); ++l) {
            if (c.slot_ticket[l] >= 0) continue;
            const CgStream::Pending pq = c.queue.front();
            c.queue.pop_front();
            c.slot_ticket[l] = pq.ticket;
            c.slot_row[l] = pq.row;
            c.slot_g[l] = pq.gidx;
            c.init_h.push_back((int)l);
            ++c.occupied;
        }
        if (!c.init_h.empty()) {
            HIPCHK(hipMemcpyAsync(c.init.p, c.init_h.data(), c.init_h.size() * 4, hipMemcpyHostToDevice, c.st));
            HIPCHK(launch_cg_init(a, (int64_t)c.init_h.size(), c.st));
            if ((rc = regroup())) return rc;
        }
        if (c.occupied == 0) break;
        for (int q = 0; q < ctx->opt_check; ++q) {
            HIPCHK(launch_cg_apply_mfma(a, a.p, c.Y.as<double>(), ctx->SR, c.G.d_work.as<int4>(), c.G.nwork,
                                        c.G.d_perm.as<int>(), ctx->max_R, c.st));
            HIPCHK(launch_cg_update2(a, c.Y.as<double>(), ctx->SR, pos, c.st));
        }
        ++c.groups_run;
        HIPCHK(hipMemcpyAsync(c.act.data(), a.active, c.S * 4, hipMemcpyDeviceToHost, c.st));
        HIPCHK(hipStreamSynchronize(c.st));
        // finished realizations leave their slots for their requests' buffers
        std::vector<int> gs;
        std::vector<double*> gl;
        std::vector<double*> gr;
        std::vector<int32_t*> gi, gt;
        for (int64_t l = 0; l < c.S; ++l) {
            if (c.slot_ticket[l] < 0 || c.act[l]) continue;
            CgStream::Req& rq = c.reqs[c.slot_ticket[l]];
            const int row = c.slot_row[l];
            gs.push_back((int)l);
            gl.push_back(rq.lam + (int64_t)row * M);
            gi.push_back(rq.it ? rq.it + row : nullptr);
            gr.push_back(rq.rel ? rq.rel + row : nullptr);
            gt.push_back(rq.st ? rq.st + row : nullptr);
            if (--rq.remaining == 0) finished.push_back(c.slot_ticket[l]);
            c.slot_ticket[l] = -1;
            c.slot_row[l] = -1;
            --c.occupied;
        }
        if (!gs.empty()) {
            const size_t k = gs.size();
            HIPCHK(hipMemcpyAsync(c.g_slot.p, gs.data(), k * 4, hipMemcpyHostToDevice, c.st));
            HIPCHK(hipMemcpyAsync(c.g_lam.p, gl.data(), k * 8, hipMemcpyHostToDevice, c.st));
            HIPCHK(hipMemcpyAsync(c.g_it.p, gi.data(), k * 8, hipMemcpyHostToDevice, c.st));
            HIPCHK(hipMemcpyAsync(c.g_rel.p, gr.data(), k * 8, hipMemcpyHostToDevice, c.st));
            HIPCHK(hipMemcpyAsync(c.g_st.p, gt.data(), k * 8, hipMemcpyHostToDevice, c.st));
            HIPCHK(launch_stream_gather(c.lam.as<double>(), M, c.g_slot.as<int>(), c.g_lam.as<double*>(),
                                        c.iters.as<int32_t>(), c.relres.as<double>(), c.status.as<int32_t>(),
                                        c.g_it.as<int32_t*>(), c.g_rel.as<double*>(), c.g_st.as<int32_t*>(), (int)k,
                                        c.st));
            HIPCHK(hipStreamSynchronize(c.st));   // the host lists are rebuilt at the next check
            // the freed slots are refilled at the next admission; when nothing
            // waits, the operator shrinks to the realizations still iterating
            if (c.queue.empty() && c.occupied > 0 && c.occupied < 0.75 * c.in_work && (rc = regroup())) return rc;
        }
    }
    int64_t nd = 0;
    for (int64_t t : finished) {
        if (nd < cap) done[nd] = t;
        ++nd;
        c.reqs.erase(t);
    }
    *n_done = std::min(nd, cap);
    if (in_flight) *in_flight = c.occupied + (int64_t)c.queue.size();
    if (nd > cap) return fail(ctx, SDMM_EINVAL, "done capacity too small (tickets beyond it were dropped)");
    return SDMM_OK;
}

int impl_stream_close(Prob* ctx, int64_t sid) {
    CgStream* c;
    int rc;
    if (!ctx) return SDMM_EINVAL;
    if ((rc = find_stream(ctx, sid, &c))) return rc;
    HIPCHK(hipSetDevice(ctx->device));
    HIPCHK(hipStreamSynchronize(c->st));
    ctx->streams.erase(sid);
    return SDMM_OK;
}

int impl_autotune(Prob* ctx, int64_t n, const int64_t* gidx, double rtol, int32_t max_iter, void* stream,
                  int64_t* chunk_out) {
    if (ctx && ctx->method != SDMM_METHOD_STOCHASTIC)
        return fail(ctx, SDMM_ESTATE, "needs a stochastic basis (Method S3); this problem was built for Method S1 or S2");
    if (!ctx) return SDMM_EINVAL;
    if (ctx->host_only) return fail(ctx, SDMM_ESTATE, "context has no device");
    if (!ctx->basis_built) return fail(ctx, SDMM_ESTATE, "basis not built");
    if (n < 1 || !gidx || !(rtol > 0) || max_iter < 1) return fail(ctx, SDMM_EINVAL, "invalid arguments");
    if (n > 2147483647LL) return fail(ctx, SDMM_EINVAL, "batch too large");
    HIPCHK(hipSetDevice(ctx->device));
    hipStream_t user = (hipStream_t)stream;
    hipStream_t st = work_stream(ctx, user);
    HIPCHK(hipEventRecord(ctx->ev[5], user));
    HIPCHK(hipStreamWaitEvent(st, ctx->ev[5], 0));
    int rc;
    if ((rc = check_indices(ctx, gidx, n, st))) return rc;
    // the sample: the first realizations of the batch; candidate slot counts:
    // all of it, 1024 .. 8192 in steps of 512 below its size, and the
    // cache-budget default
    const int64_t ns = std::min<int64_t>(n, 16384);
    const int64_t saved = ctx->opt_chunk;
    ctx->opt_chunk = 0;
    std::vector<int64_t> cand{ns};
    for (int64_t c = 1024; c <= 8192; c += 512)
        if (c < ns) cand.push_back(c);
    cand.push_back(chunk_size(ctx, ns));
    std::sort(cand.begin(), cand.end());
    cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
    if ((rc = ensure_workspace(ctx, cand.back()))) {
        ctx->opt_chunk = saved;
        return rc;
    }
    DevBuf lam;
    if ((rc = alloc(ctx, lam, (size_t)ns * ctx->P.M * 8))) {
        ctx->opt_chunk = saved;
        return rc;
    }
    const sdmm_counters saved_counters = ctx->counters;
    double best = 1e300;
    int64_t best_c = cand.back();
    for (int64_t c : cand) {
        // the whole sample through CG with c slots: the final drain and
        // cache residency are both in the measurement
        int64_t tot = 0;
        bool bad = false, brk = false;
        HIPCHK(hipStreamSynchronize(st));
        const auto t0 = std::chrono::steady_clock::now();
        rc = solve_batch(ctx, ns, c, gidx, rtol, max_iter, lam.as<double>(), nullptr, nullptr, nullptr, st, tot, bad,
                         brk);
        if (rc) {
            ctx->opt_chunk = saved;
            ctx->counters = saved_counters;
            return rc;
        }
        HIPCHK(hipStreamSynchronize(st));
        const double t = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (t < best) {
            best = t;
            best_c = c;
        }
    }
    ctx->counters = saved_counters;
    ctx->opt_chunk = best_c;
    if (chunk_out) *chunk_out = best_c;
    HIPCHK(hipEventRecord(ctx->ev[4], st));
    HIPCHK(hipStreamWaitEvent(user, ctx->ev[4], 0));
    return SDMM_OK;
}

// chunk_override > 0: that many realizations per pass; alpha_ready: the
// FETI coefficients of the (single) pass are already in w_alpha
int accumulate_core(Prob* ctx, int64_t n, const int64_t* grp_idx, const int64_t* w_idx, const double* lambda,
                    const double* weights, hipStream_t st, int64_t chunk_override, bool alpha_ready) {
    int rc;
    const int64_t chunk = chunk_override > 0 ? chunk_override : chunk_size(ctx, n);
    if ((rc = ensure_workspace(ctx, chunk))) return rc;
    const int M = ctx->P.M;
    const BasisView* v = ctx->view;
    for (int64_t c0 = 0; c0 < n; c0 += chunk) {
        const int64_t cn = std::min(chunk, n - c0);
        const int64_t* g = grp_idx + c0;
        const double* lam = lambda + c0 * M;
        if ((rc = fetch_gidx(ctx, g, cn, st))) return rc;
        Groups& G = ctx->grp[0];
        if ((rc = build_groups(ctx, G, cn, nullptr, ctx->h_gidx.data(), st))) return rc;
        CgArgs a = cg_args(ctx, cn, g, const_cast<double*>(lam));
        if (ctx->P.n_kernel > 0 && !alpha_ready) {
            HIPCHK(launch_cg_apply_mfma(a, lam, ctx->w_Y.as<double>(), ctx->SR,
                                        G.d_work.as<int4>(), G.nwork, G.d_perm.as<int>(), ctx->max_R, st));
            HIPCHK(launch_gather_global(ctx->w_Y.as<double>(), ctx->SR, ctx->d_pos.as<int>(), M, cn,
                                        ctx->w_Slam.as<double>(), st));
            HIPCHK(launch_alpha(a, ctx->w_Slam.as<double>(), ctx->w_alpha.as<double>(), st));
        }
        if (ctx->d_part.bytes < (size_t)G.part_total * 8 && (rc = alloc(ctx, ctx->d_part, G.part_total * 8)))
            return rc;
        MomArgs m{};
        m.n = cn;
        m.M = M;
        m.nsub = (int)ctx->P.subs.size();
        m.nregion = ctx->P.n_region;
        m.nker = ctx->P.n_kernel;
        m.gidx = w_idx ? w_idx + c0 : nullptr;
        m.g2l = ctx->d_g2l.as<int32_t>();
        m.weights = weights ? weights + c0 : nullptr;
        m.colloc_w = ctx->d_weights.as<double>();
        m.lam = lam;
        m.sub_R = ctx->d_sub_R.as<int>();
        m.sub_dof_ptr = ctx->d_sub_dof_ptr.as<int64_t>();
        m.sub_dofs = ctx->d_sub_dofs.as<int64_t>();
        m.sub_region = ctx->d_sub_region.as<int>();
        m.sub_ker = ctx->d_sub_ker.as<int>();
        m.sub_Gcol = ctx->d_sub_Gcol.as<int>();
        m.sub_Abase = v ? v->d_sub_Abase.as<int64_t>() : ctx->d_sub_Abase.as<int64_t>();
        m.sub_nlocal = ctx->d_sub_nlocal.as<int>();
        m.alpha = ctx->w_alpha.as<double>();
        m.acc = ctx->d_acc.as<double>();
        m.lam1 = ctx->d_lam1.as<double>();
        m.lam2 = ctx->d_lam2.as<double>();
        m.wsum = ctx->d_wsum.as<double>();
        const int npairs = (int)(v ? v->pair_sub.size() : ctx->pair_sub.size());
        HIPCHK(launch_accumulate_chunks(m, G.d_awork.as<int4>(), G.nawork, G.d_perm.as<int>(),
                                        G.d_slot.as<int64_t>(), ctx->d_part.as<double>(),
                                        v ? v->d_pair_sub.as<int>() : ctx->d_pair_sub.as<int>(),
                                        v ? v->d_pair_k.as<int>() : ctx->d_pair_k.as<int>(), G.d_item0.as<int>(),
                                        npairs, ctx->max_ext, st));
        HIPCHK(hipStreamSynchronize(st));  // the group tables are rebuilt by the next chunk
    }
    ctx->moments_final = false;
    return SDMM_OK;
}

int impl_accumulate_moments(Prob* ctx, int64_t n, const int64_t* gidx, const double* y, const double* lambda,
                            const double* weights, void* stream) {
    if (!ctx) return SDMM_EINVAL;
    ctx->view = nullptr;
    const bool det = ctx->method == SDMM_METHOD_DETERMINISTIC;
    const bool s1 = ctx->method == SDMM_METHOD_PER_ITERATION;
    if (n > 0 && !gidx && y && !det && !s1)
        return fail(ctx, SDMM_EINVAL, "off-grid points need Method S2 or S1 (a stochastic basis exists only on the grid)");
    if (ctx->host_only) return fail(ctx, SDMM_ESTATE, "context has no device");
    if (!ctx->basis_built) return fail(ctx, SDMM_ESTATE, "basis not built");
    if (n < 0 || (n > 0 && ((!gidx && !((det || s1) && y && weights)) || !lambda)))
        return fail(ctx, SDMM_EINVAL, "invalid arguments (off-grid points need weights)");
    if (n == 0) return SDMM_OK;
    HIPCHK(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    int rc;
    if (!det && !s1) {
        if ((rc = check_indices(ctx, gidx, n, st))) return rc;
        return accumulate_core(ctx, n, gidx, gidx, lambda, weights, st);
    }
    // Methods S2 and S1: the realizations of the last solve, with their own
    // bases (S2) or factors (S1)
    DetBatch& D = ctx->det;
    std::vector<double> pts;
    if ((rc = det_points(ctx, n, gidx, y, st, pts))) return rc;
    if (!D.valid || n != D.n || pts != D.y)
        return fail(ctx, SDMM_ESTATE, "the local problems exist only for the points of the last solve");
    if (s1) return s1_accumulate(ctx, n, gidx, lambda, weights, st);
    const int64_t a_end = D.A_base + (int64_t)(D.view.pair_sub.size() - ctx->P.stokes.size()) * 0;
    (void)a_end;
    int64_t a_n = 0;
    for (auto& h : ctx->P.darcy) a_n += n * ((int64_t)h.R + (int64_t)h.R * h.R);
    HIPCHK(hipMemsetAsync(ctx->d_acc.as<double>() + D.A_base, 0, a_n * 8, st));
    ctx->view = &D.view;
    rc = accumulate_core(ctx, n, D.d_pos.as<int64_t>(), gidx, lambda, weights, st);
    ctx->view = nullptr;
    if (rc) return rc;
    // expand this batch's Darcy moments with its own responses and add them
    const int64_t f1 = ctx->field_size[1], f2 = ctx->field_size[2];
    double* tmp = D.d_tmp.as<double>();
    DarcyTables t = darcy_tables(ctx);
    t.units = D.d_units.as<UnitDev>();
    t.order = D.d_order.as<int>();
    t.xi = D.d_xi.as<double>();
    HIPCHK(launch_darcy_moments_impl(t, D.d_unit_of_dk.as<int>(), D.d_dnlocal.as<int>(), (int)ctx->P.darcy.size(),
                                     ctx->max_nout_d, (int)n, D.d_dAbase.as<int64_t>(), ctx->d_acc.as<double>(),
                                     D.d_X.as<double>(), ctx->max_Rd, ctx->d_cell_out.as<int64_t>(),
                                     ctx->d_edge_out.as<int64_t>(), tmp, tmp + f1, tmp + 2 * f1, tmp + 2 * f1 + f2,
                                     st));
    HIPCHK(launch_add_inplace(D.d_sum.as<double>(), tmp, 2 * (f1 + f2), st));
    HIPCHK(hipStreamSynchronize(st));
    return SDMM_OK;
}

int impl_reset_moments(Prob* ctx) {
    if (!ctx) return SDMM_EINVAL;
    if (ctx->host_only) return fail(ctx, SDMM_ESTATE, "context has no device");
    if (!ctx->have_problem) return fail(ctx, SDMM_ESTATE, "no problem set");
    HIPCHK(hipSetDevice(ctx->device));
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(hipMemset(ctx->d_acc.p, 0, ctx->d_acc.bytes));
    HIPCHK(hipMemset(ctx->d_lam1.p, 0, ctx->d_lam1.bytes));
    HIPCHK(hipMemset(ctx->d_lam2.p, 0, ctx->d_lam2.bytes));
    HIPCHK(hipMemset(ctx->d_wsum.p, 0, 8));
    if (ctx->det.d_sum.p) HIPCHK(hipMemset(ctx->det.d_sum.p, 0, ctx->det.d_sum.bytes));
    ctx->moments_final = false;
    return SDMM_OK;
}

// Expansion of the reduced moments to the fine fields (Section 2 moments of
// the Darcy and Stokes responses): E[u] = Phi a and E[u^2] = diag(Phi Mc Phi^T)
// per (subdomain, local realization), into the device field buffers.
int finalize_moments(Prob* ctx, hipStream_t st) {
    double* base = ctx->d_mom.as<double>();
    double* p1 = base;
    double* p2 = p1 + ctx->field_size[1];
    double* u1 = p2 + ctx->field_size[1];
    double* u2 = u1 + ctx->field_size[2];
    double* su1 = u2 + ctx->field_size[2];
    double* su2 = su1 + ctx->field_size[3];
    double* sp1 = su2 + ctx->field_size[3];
    double* sp2 = sp1 + ctx->field_size[4];
    HIPCHK(hipEventRecord(ctx->ev[6], st));
    if (ctx->method != SDMM_METHOD_STOCHASTIC) {
        // Methods S2 and S1: the Darcy moments were expanded batch by batch
        const size_t nd = (size_t)2 * (ctx->field_size[1] + ctx->field_size[2]);
        if (ctx->det.d_sum.p)
            HIPCHK(hipMemcpyAsync(p1, ctx->det.d_sum.p, nd * 8, hipMemcpyDeviceToDevice, st));
        else
            HIPCHK(hipMemsetAsync(p1, 0, nd * 8, st));
    } else {
        DarcyTables t = darcy_tables(ctx);
        HIPCHK(launch_darcy_moments_impl(t, ctx->d_unit_of_dk.as<int>(), ctx->d_dnlocal.as<int>(),
                                         (int)ctx->P.darcy.size(), ctx->max_nout_d, ctx->max_units_per_d,
                                         ctx->d_dAbase.as<int64_t>(), ctx->d_acc.as<double>(), ctx->d_X.as<double>(),
                                         ctx->max_Rd, ctx->d_cell_out.as<int64_t>(), ctx->d_edge_out.as<int64_t>(),
                                         p1, p2, u1, u2, st));
    }
    HIPCHK(launch_stokes_moments_impl(ctx->d_sdev.as<StokesDev>(), (int)ctx->sdev.size(), ctx->max_nout_s,
                                      ctx->d_sAbase.as<int64_t>(), ctx->d_acc.as<double>(), ctx->d_wsum.as<double>(),
                                      ctx->d_U.as<double>(), ctx->d_P.as<double>(), ctx->d_Z.as<double>(),
                                      ctx->d_u_out.as<int64_t>(), ctx->d_p_out.as<int64_t>(), ctx->max_ext, su1, su2,
                                      sp1, sp2, st));
    HIPCHK(hipEventRecord(ctx->ev[7], st));
    ctx->moments_final = true;
    ctx->moments_timed = true;
    return SDMM_OK;
}

int impl_finalize_moments(Prob* ctx, void* stream) {
    if (!ctx) return SDMM_EINVAL;
    if (ctx->host_only) return fail(ctx, SDMM_ESTATE, "context has no device");
    if (!ctx->basis_built) return fail(ctx, SDMM_ESTATE, "basis not built");
    HIPCHK(hipSetDevice(ctx->device));
    return finalize_moments(ctx, (hipStream_t)stream);
}

int impl_get_moments(Prob* ctx, int field, double* mean, double* var, int64_t cap) {
    if (!ctx || !mean || !var) return fail(ctx, SDMM_EINVAL, "null argument");
    if (!ctx->basis_built) return fail(ctx, SDMM_ESTATE, "basis not built");
    if (field < 0 || field > 4) return fail(ctx, SDMM_EINVAL, "bad field");
    if (cap < ctx->field_size[field]) return fail(ctx, SDMM_EINVAL, "output capacity too small");
    HIPCHK(hipSetDevice(ctx->device));
    HIPCHK(hipDeviceSynchronize());
    const int64_t n = ctx->field_size[field];
    std::vector<double> m1(n), m2(n);
    if (field == SDMM_FIELD_LAMBDA) {
        HIPCHK(hipMemcpy(m1.data(), ctx->d_lam1.p, n * 8, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(m2.data(), ctx->d_lam2.p, n * 8, hipMemcpyDeviceToHost));
    } else {
        if (!ctx->moments_final) {
            int rc = finalize_moments(ctx, 0);
            if (rc) return rc;
            HIPCHK(hipDeviceSynchronize());
        }
        double* base = ctx->d_mom.as<double>();
        int64_t off = 0;
        for (int f = 1; f < field; ++f) off += 2 * ctx->field_size[f];
        HIPCHK(hipMemcpy(m1.data(), base + off, n * 8, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(m2.data(), base + off + n, n * 8, hipMemcpyDeviceToHost));
    }
    for (int64_t q = 0; q < n; ++q) {
        mean[q] = m1[q];
        var[q] = m2[q] - m1[q] * m1[q];
    }
    return SDMM_OK;
}

int impl_get_counters(Prob* ctx, sdmm_counters* out) {
    if (!ctx || !out) return fail(ctx, SDMM_EINVAL, "null argument");
    if (ctx->host_only) {
        *out = ctx->counters;
        return SDMM_OK;
    }
    HIPCHK(hipSetDevice(ctx->device));
    HIPCHK(hipDeviceSynchronize());
    float ms = 0;
    if (ctx->basis_built) {
        if (hipEventElapsedTime(&ms, ctx->ev[0], ctx->ev[1]) == hipSuccess) ctx->counters.ms_basis_darcy = ms;
        if (hipEventElapsedTime(&ms, ctx->ev[0], ctx->ev[8]) == hipSuccess) ctx->counters.ms_basis_stokes = ms;
        if (hipEventElapsedTime(&ms, ctx->ev[0], ctx->ev[2]) == hipSuccess) ctx->counters.ms_basis_build = ms;
        if (ctx->moments_timed && hipEventElapsedTime(&ms, ctx->ev[6], ctx->ev[7]) == hipSuccess)
            ctx->counters.ms_moments = ms;
        if (ctx->built_precision == SDMM_PREC_MIXED && ctx->d_refine.p) {
            double mr;
            int steps;
            HIPCHK(hipMemcpy(&mr, ctx->d_refine.p, 8, hipMemcpyDeviceToHost));
            HIPCHK(hipMemcpy(&steps, ctx->d_refine.as<char>() + 8, 4, hipMemcpyDeviceToHost));
            ctx->counters.max_refine_residual = mr;
            ctx->counters.refinement_steps = steps;
        }
    }
    *out = ctx->counters;
    return SDMM_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// The C ABI: a context is a device, an optional allocator and a table of
// problems; every call on a problem names its id.
// ---------------------------------------------------------------------------
struct sdmm_ctx {
    int device = 0;
    bool host_only = false;
    bool have_alloc = false;
    sdmm_alloc alloc{};
    std::string err;
    std::map<int64_t, std::unique_ptr<Prob, int (*)(Prob*)>> probs;
    int64_t next_id = 1;
};

namespace {

int ctx_fail(sdmm_ctx* c, int code, const std::string& msg) {
    if (c) c->err = msg;
    return code;
}

// the problem `id` of c, or an error
int find(sdmm_ctx* c, int64_t id, Prob** out) {
    if (!c) return SDMM_EINVAL;
    auto it = c->probs.find(id);
    if (it == c->probs.end()) return ctx_fail(c, SDMM_EINVAL, "unknown problem id " + std::to_string(id));
    *out = it->second.get();
    return SDMM_OK;
}

// a call's status, with the problem's message copied to the context on failure
int relay(sdmm_ctx* c, Prob* p, int rc) {
    if (rc != SDMM_OK) c->err = p->err.empty() ? "error " + std::to_string(rc) : p->err;
    return rc;
}

#define WITH_PROB(call)                          \
    do {                                         \
        Prob* p_ = nullptr;                      \
        int rc_ = find(ctx, id, &p_);            \
        if (rc_) return rc_;                     \
        p_->err.clear();                         \
        return relay(ctx, p_, call);             \
    } while (0)

}  // namespace

extern "C" {

int sdmm_create(int device, const sdmm_alloc* alloc, sdmm_ctx** out) {
    if (!out) return SDMM_EINVAL;
    *out = nullptr;
    if (alloc && (!alloc->alloc || !alloc->release)) return SDMM_EINVAL;
    if (device != -1) {
        int count = 0;
        if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return SDMM_EINVAL;
        if (hipSetDevice(device) != hipSuccess) return SDMM_EDEVICE;
        // the allocation-free entry point's scratch on this device (once per device)
        if (noalloc_scratch_setup(device) != hipSuccess) return SDMM_EDEVICE;
    }
    sdmm_ctx* c = new (std::nothrow) sdmm_ctx();
    if (!c) return SDMM_ENOMEM;
    c->device = device;
    c->host_only = device == -1;
    if (alloc) {
        c->alloc = *alloc;
        c->have_alloc = true;
    }
    *out = c;
    return SDMM_OK;
}

int sdmm_destroy(sdmm_ctx* ctx) {
    if (!ctx) return SDMM_EINVAL;
    ctx->probs.clear();
    delete ctx;
    return SDMM_OK;
}

const char* sdmm_last_error(const sdmm_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int sdmm_set_problem(sdmm_ctx* ctx, const sdmm_problem* p, int64_t* problem_id) {
    if (!ctx) return SDMM_EINVAL;
    if (!p || !problem_id) return ctx_fail(ctx, SDMM_EINVAL, "null argument");
    Prob* q = nullptr;
    int rc = impl_create(ctx->device, ctx->have_alloc ? &ctx->alloc : nullptr, &q);
    if (rc) return ctx_fail(ctx, rc, "could not create the problem's device state");
    std::unique_ptr<Prob, int (*)(Prob*)> holder(q, impl_destroy);
    rc = impl_set_problem(q, p);
    if (rc) return relay(ctx, q, rc);
    const int64_t id = ctx->next_id++;
    ctx->probs.emplace(id, std::move(holder));
    *problem_id = id;
    return SDMM_OK;
}

int sdmm_release_problem(sdmm_ctx* ctx, int64_t id) {
    Prob* p = nullptr;
    int rc = find(ctx, id, &p);
    if (rc) return rc;
    ctx->probs.erase(id);
    return SDMM_OK;
}

int sdmm_get_sizes(sdmm_ctx* ctx, int64_t id, sdmm_sizes* o) {
    if (ctx && !o) return ctx_fail(ctx, SDMM_EINVAL, "null argument");
    WITH_PROB(impl_get_sizes(p_, o));
}

int sdmm_get_index_maps(sdmm_ctx* ctx, int64_t id, int kind, int64_t* out, int64_t cap, int64_t* n_out) {
    WITH_PROB(impl_get_index_map(p_, kind, out, cap, n_out));
}

int sdmm_get_collocation(sdmm_ctx* ctx, int64_t id, double* points, double* weights) {
    WITH_PROB(impl_get_collocation(p_, points, weights));
}

int sdmm_get_kl(sdmm_ctx* ctx, int64_t id, int region, double* lam, int32_t* modes) {
    WITH_PROB(impl_get_kl(p_, region, lam, modes));
}

int sdmm_build_flux_basis(sdmm_ctx* ctx, int64_t id, int method, int precision, void* stream) {
    WITH_PROB(impl_build_flux_basis(p_, method, precision, stream));
}

int sdmm_get_basis(sdmm_ctx* ctx, int64_t id, int sub, int k, double* S, int64_t ld) {
    WITH_PROB(impl_get_basis(p_, sub, k, S, ld));
}

int sdmm_get_interface_data(sdmm_ctx* ctx, int64_t id, double* g, double* G) {
    WITH_PROB(impl_get_interface_data(p_, g, G));
}

int sdmm_solve_interface(sdmm_ctx* ctx, int64_t id, int64_t n, const int64_t* gidx, const double* y, double rtol,
                         int32_t max_iter, double* lambda, int32_t* iters, double* relres, int32_t* status,
                         void* stream) {
    WITH_PROB(impl_solve_interface(p_, n, gidx, y, rtol, max_iter, lambda, iters, relres, status, stream));
}

int sdmm_solve_interface_noalloc(sdmm_ctx* ctx, int64_t id, int64_t n, const int64_t* gidx, double rtol,
                                 int32_t max_iter, double* lambda, int32_t* iters, double* relres, int32_t* status,
                                 void* stream) {
    WITH_PROB(impl_solve_interface_noalloc(p_, n, gidx, rtol, max_iter, lambda, iters, relres, status, stream));
}

int sdmm_stream_open(sdmm_ctx* ctx, int64_t id, int64_t slots, double rtol, int32_t max_iter, void* stream,
                     int64_t* sid) {
    WITH_PROB(impl_stream_open(p_, slots, rtol, max_iter, stream, sid));
}
int sdmm_stream_submit(sdmm_ctx* ctx, int64_t id, int64_t sid, int64_t n, const int64_t* gidx, double* lambda,
                       int32_t* iters, double* relres, int32_t* status, int64_t* ticket) {
    WITH_PROB(impl_stream_submit(p_, sid, n, gidx, lambda, iters, relres, status, ticket));
}
int sdmm_stream_run(sdmm_ctx* ctx, int64_t id, int64_t sid, int32_t max_groups, int64_t* done, int64_t cap,
                    int64_t* n_done, int64_t* in_flight) {
    WITH_PROB(impl_stream_run(p_, sid, max_groups, done, cap, n_done, in_flight));
}
int sdmm_stream_close(sdmm_ctx* ctx, int64_t id, int64_t sid) { WITH_PROB(impl_stream_close(p_, sid)); }

int sdmm_noalloc_scratch_bytes(int64_t* bytes) {
    if (!bytes) return SDMM_EINVAL;
    *bytes = (int64_t)kNoAllocScratchBytes;
    return SDMM_OK;
}

int sdmm_accumulate_moments(sdmm_ctx* ctx, int64_t id, int64_t n, const int64_t* gidx, const double* y,
                            const double* lambda, const double* weights, void* stream) {
    WITH_PROB(impl_accumulate_moments(p_, n, gidx, y, lambda, weights, stream));
}

int sdmm_get_moments(sdmm_ctx* ctx, int64_t id, int field, double* mean, double* var, int64_t cap) {
    WITH_PROB(impl_get_moments(p_, field, mean, var, cap));
}

int sdmm_reset_moments(sdmm_ctx* ctx, int64_t id) { WITH_PROB(impl_reset_moments(p_)); }
int sdmm_finalize_moments(sdmm_ctx* ctx, int64_t id, void* stream) { WITH_PROB(impl_finalize_moments(p_, stream)); }

int sdmm_set_option(sdmm_ctx* ctx, int64_t id, int option, int64_t value) {
    WITH_PROB(impl_set_option(p_, option, value));
}

int sdmm_autotune(sdmm_ctx* ctx, int64_t id, int64_t n, const int64_t* gidx, double rtol, int32_t max_iter,
                  void* stream, int64_t* chunk_out) {
    WITH_PROB(impl_autotune(p_, n, gidx, rtol, max_iter, stream, chunk_out));
}

int sdmm_get_counters(sdmm_ctx* ctx, int64_t id, sdmm_counters* out) { WITH_PROB(impl_get_counters(p_, out)); }

}  // extern "C"
