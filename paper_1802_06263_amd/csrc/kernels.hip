// HIP kernels of the stochastic multiscale flux basis library (gfx950).
//
//   darcy_basis_*      Method S3 pre-computation loop for Darcy subdomains
//                      (Section 5.4): per (subdomain, local realization) unit,
//                      K = exp(Y) from the KL expansion (eq. KLapprox), the
//                      RT0-Q0 cell-centred operator, its blocked band LDL^T
//                      factor, the solves for every mortar basis function
//                      (eqs. starDproblem1-2) and the flux basis S_{H,i}^{(k)}
//                      (darcy_blocked.inc).
//   stokes_*           the same for Stokes subdomains (eqs. starSproblem1-2,
//                      barSproblem1-2) with a tiled band LDL^T of the
//                      Taylor-Hood saddle matrix.
//   cg_*               CG on S_H lambda = g_H (Section 5.1) batched over
//                      collocation points, S_H applied as linear combinations
//                      of the basis (Section 5.3).
//   accumulate / *_moments   weighted moments (Section 2, Step 6 of S3).
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <cmath>
#include <mutex>

#include "kernels.hpp"
#include "../../include/sdmm.h"

namespace sdmm {

namespace {

constexpr int kThreads = 256;
constexpr int kTile = 64;

__device__ inline double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Deterministic block sum (fixed order for a fixed block size).  `red` holds
// at least blockDim.x / 64 doubles.  The result is returned to every thread.
__device__ inline double block_sum(double v, double* red) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double s = 0.0;
    const int nw = (blockDim.x + 63) >> 6;
    for (int k = 0; k < nw; ++k) s += red[k];
    __syncthreads();
    return s;
}

__device__ inline int cell_of_internal(int c, int nx, int ny, int swap) {
    if (!swap) return c;
    const int ix = c / ny, iy = c - ix * ny;
    return iy * nx + ix;
}

__device__ inline int internal_of_cell(int cell, int nx, int ny, int swap) {
    if (!swap) return cell;
    const int iy = cell / nx, ix = cell - iy * nx;
    return ix * ny + iy;
}

__device__ inline double darcy_K(const DarcyTables& t, const DarcyDev& D, const double* xi, int cell) {
    double y = D.mean_logk;
    const double* phi = t.phi + D.off_phi;
    for (int s = 0; s < D.nterm; ++s) y += xi[s] * phi[(int64_t)s * D.N + cell];
    return exp(y);
}

// Transmissibilities of one unit (the RT0-Q0 operator with trapezoidal mass):
//   Tf[c]  between internal cells c and c+1 (0 at the end of a line)
//   Ts[c]  between internal cells c and c+b (0 on the last line)
//   Tb[c]  sum of Dirichlet / mortar boundary-edge terms of cell c
//   Tm[e]  the term of mortar edge e
__device__ void darcy_transmissibilities(const DarcyTables& t, const DarcyDev& D, const double* xi, double* Ksc,
                                         double* Tf, double* Ts, double* Tb, double* Tm) {
    const int N = D.N, b = D.b;
    for (int c = threadIdx.x; c < N; c += blockDim.x) Ksc[c] = darcy_K(t, D, xi, cell_of_internal(c, D.nx, D.ny, D.swap));
    __syncthreads();
    const double nu = D.nu;
    // edges along the fast direction have length h_slow and normal spacing h_fast
    const double hf = D.swap ? D.hy : D.hx, hs = D.swap ? D.hx : D.hy;
    for (int c = threadIdx.x; c < N; c += blockDim.x) {
        const double kc = Ksc[c];
        double tf = 0.0, ts = 0.0;
        if ((c % b) != b - 1) tf = hs / (nu * (0.5 * hf) * (1.0 / kc + 1.0 / Ksc[c + 1]));
        if (c + b < N) ts = hf / (nu * (0.5 * hs) * (1.0 / kc + 1.0 / Ksc[c + b]));
        Tf[c] = tf;
        Ts[c] = ts;
        const int cell = cell_of_internal(c, D.nx, D.ny, D.swap);
        double tb = 0.0;
        for (int q = 0; q < 2; ++q) {
            const int e = t.cell_be[D.off_cellbe + 2 * cell + q];
            if (e < 0) continue;
            const int kind = t.be_kind[D.off_be + e];
            if (kind == 2) continue;
            const double T = 2.0 * t.be_len[D.off_be + e] * kc / (nu * t.be_hperp[D.off_be + e]);
            tb += T;
            if (kind == 0) Tm[t.be_medge[D.off_be + e]] = T;
        }
        Tb[c] = tb;
    }
    __syncthreads();
}

}  // namespace

#include "darcy_blocked.inc"
#include "kl.inc"

// ---------------------------------------------------------------------------
// Stokes: tiled band LDL^T.  Block column J holds tiles I = J .. J + w, each
// 64 x 64 column-major; tile (I, J) at off_tiles + (J (w+1) + I - J) 4096.
// ---------------------------------------------------------------------------
__device__ inline double* tile_ptr(double* base, const StokesDev& s, int I, int J) {
    return base + s.off_tiles + ((int64_t)J * (s.w + 1) + (I - J)) * (kTile * kTile);
}
__device__ inline const double* tile_ptr(const double* base, const StokesDev& s, int I, int J) {
    return base + s.off_tiles + ((int64_t)J * (s.w + 1) + (I - J)) * (kTile * kTile);
}

__global__ void stokes_scatter_kernel(const StokesDev* sd, const int* tr_sub, const int* tr_r, const int* tr_c,
                                      const double* tr_v, int64_t ntrip, double* tiles) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= ntrip) return;
    const StokesDev s = sd[tr_sub[q]];
    const int r = tr_r[q], c = tr_c[q];
    const int I = r / kTile, J = c / kTile;
    double* T = tile_ptr(tiles, s, I, J);
    T[(c % kTile) * kTile + (r % kTile)] = tr_v[q];
}

__global__ void stokes_pad_kernel(const StokesDev* sd, double* tiles) {
    const StokesDev s = sd[blockIdx.y];
    const int J = blockIdx.x;
    if (J >= s.nblk) return;
    for (int d = threadIdx.x; d < kTile; d += blockDim.x) {
        const int row = J * kTile + d;
        if (row >= s.nband) tile_ptr(tiles, s, J, J)[d * kTile + d] = 1.0;
    }
}

hipError_t launch_stokes_scatter(const StokesDev* sd, int ns, const int* tr_sub, const int* tr_r, const int* tr_c,
                                 const double* tr_v, int64_t ntrip, double* tiles, hipStream_t stream) {
    if (ntrip <= 0) return hipSuccess;
    hipLaunchKernelGGL(stokes_scatter_kernel, dim3((unsigned)((ntrip + 255) / 256)), dim3(256), 0, stream, sd, tr_sub,
                       tr_r, tr_c, tr_v, ntrip, tiles);
    return hipGetLastError();
}

hipError_t launch_stokes_pad_identity(const StokesDev* sd, int ns, int max_nblk, double* tiles, hipStream_t stream) {
    if (ns <= 0) return hipSuccess;
    hipLaunchKernelGGL(stokes_pad_kernel, dim3(max_nblk, ns), dim3(64), 0, stream, sd, tiles);
    return hipGetLastError();
}

#include "stokes_tiled.inc"

__global__ void add_inplace_kernel(double* __restrict__ x, const double* __restrict__ d, int64_t n) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
        x[q] += d[q];
}

__global__ void fill_zero_kernel(double* __restrict__ x, int64_t n) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
        x[q] = 0.0;
}

hipError_t launch_fill_zero(double* x, int64_t n, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, x, n);
    return hipGetLastError();
}

hipError_t launch_add_inplace(double* x, const double* d, int64_t n, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(add_inplace_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, x, d, n);
    return hipGetLastError();
}

// Scatter the band solutions to raw velocity / pressure layouts, project the
// floating subdomains' responses onto the complement of the rigid motions,
// then S = -Q U (basis columns), g += Q u_bar and the FETI traces G = Q Z.
__global__ __launch_bounds__(kThreads) void stokes_fill_kernel(const StokesDev* sd, const double* uD,
                                                               const int64_t* uD_off, double* U) {
    // velocity defaults: Dirichlet values for the complementary column, 0 otherwise
    const StokesDev s = sd[blockIdx.z];
    const int col = blockIdx.y;
    if (col >= s.ncol) return;
    double* Uc = U + s.off_U + (int64_t)col * s.nvel;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < s.nvel; q += (int64_t)gridDim.x * blockDim.x)
        Uc[q] = (col == s.R) ? uD[uD_off[blockIdx.z] + q] : 0.0;
}

__global__ __launch_bounds__(kThreads) void stokes_unpack_kernel(const StokesDev* sd, const double* rhs,
                                                                 const int* bmap, double* U, double* P) {
    const StokesDev s = sd[blockIdx.z];
    const int col = blockIdx.y;
    if (col >= s.ncol) return;
    const int64_t ld = (int64_t)s.nblk * kTile;
    double* Uc = U + s.off_U + (int64_t)col * s.nvel;
    double* Pc = P + s.off_P + (int64_t)col * s.npre;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < s.nband; q += (int64_t)gridDim.x * blockDim.x) {
        const int m = bmap[s.off_map + q];
        const double v = rhs[s.off_rhs + (int64_t)col * ld + q];
        if (m >= 0) Uc[m] = v;
        else Pc[-1 - m] = v;
    }
}

__global__ __launch_bounds__(kThreads) void stokes_project_kernel(const StokesDev* sd, const double* Z, double* U) {
    __shared__ double red[kThreads / 64];
    const StokesDev s = sd[blockIdx.y];
    const int col = blockIdx.x;
    if (col >= s.ncol || s.nker == 0) return;
    double* Uc = U + s.off_U + (int64_t)col * s.nvel;
    for (int k = 0; k < s.nker; ++k) {
        const double* z = Z + s.off_Z + (int64_t)k * s.nvel;
        double part = 0.0;
        for (int q = threadIdx.x; q < s.nvel; q += blockDim.x) part += z[q] * Uc[q];
        const double dot = block_sum(part, red);
        for (int q = threadIdx.x; q < s.nvel; q += blockDim.x) Uc[q] -= dot * z[q];
        __syncthreads();
    }
}

__global__ __launch_bounds__(kThreads) void stokes_traces_kernel(const StokesDev* sd, const int* q_ptr, const int* q_col,
                                                                 const double* q_val, const int64_t* dofs,
                                                                 const double* U, const double* Z, double* S_cache,
                                                                 double* g, double* G, int M) {
    const StokesDev s = sd[blockIdx.y];
    const int col = blockIdx.x;   // 0..R-1 basis, R complementary, R+1.. kernel columns
    if (col >= s.ncol + s.nker) return;
    const int* qp = q_ptr + s.off_q;
    for (int m = threadIdx.x; m < s.R; m += blockDim.x) {
        const double* u = (col < s.ncol) ? U + s.off_U + (int64_t)col * s.nvel : Z + s.off_Z + (int64_t)(col - s.ncol) * s.nvel;
        double v = 0.0;
        for (int q = qp[m]; q < qp[m + 1]; ++q) v += q_val[q] * u[q_col[q]];
        const int64_t gd = dofs[s.off_dofs + m];
        if (col < s.R) S_cache[s.off_S + (int64_t)col * s.R + m] = -v;
        else if (col == s.R) atomicAdd(&g[gd], v);
        else G[(int64_t)(s.off_G + col - s.ncol) * M + gd] = v;
    }
}

hipError_t launch_stokes_finish(const StokesDev* sd, int ns, int max_ncol, int max_R, const double* rhs, const int* bmap,
                                const double* uD, const int64_t* uD_off, const double* Z, const int* q_ptr,
                                const int* q_col, const double* q_val, const int64_t* dofs, double* U, double* P,
                                double* S_cache, double* g, double* G, int M, hipStream_t stream) {
    if (ns <= 0) return hipSuccess;
    hipLaunchKernelGGL(stokes_fill_kernel, dim3(64, max_ncol, ns), dim3(kThreads), 0, stream, sd, uD, uD_off, U);
    hipLaunchKernelGGL(stokes_unpack_kernel, dim3(64, max_ncol, ns), dim3(kThreads), 0, stream, sd, rhs, bmap, U, P);
    hipLaunchKernelGGL(stokes_project_kernel, dim3(max_ncol, ns), dim3(kThreads), 0, stream, sd, Z, U);
    hipLaunchKernelGGL(stokes_traces_kernel, dim3(max_ncol + 8, ns), dim3(kThreads), 0, stream, sd, q_ptr, q_col, q_val,
                       dofs, U, Z, S_cache, g, G, M);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Batched interface CG.  One workgroup per realization for the vector work;
// the operator y = sum_i R_i^T S_i^{(k_i(l))} R_i x is applied by one
// workgroup per (realization, subdomain).  Every mortar DOF receives exactly
// two contributions on a zeroed vector, so the atomic adds are order
// independent and results are bit-reproducible for any batch composition.
// ---------------------------------------------------------------------------
__device__ void feti_project_row(const CgArgs& a, double* v, double* red, double* coef) {
    // v <- v - G (G^T G)^{-1} G^T v   (coef: scratch of 2 nker doubles in LDS)
    const int nk = a.nker;
    for (int k = 0; k < nk; ++k) {
        double part = 0.0;
        for (int m = threadIdx.x; m < a.M; m += blockDim.x) part += a.G[(int64_t)k * a.M + m] * v[m];
        const double s = block_sum(part, red);
        if (threadIdx.x == 0) coef[k] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 0; k < nk; ++k) {
            double d = 0.0;
            for (int q = 0; q < nk; ++q) d += a.GtGinv[k * nk + q] * coef[q];
            coef[nk + k] = d;
        }
    }
    __syncthreads();
    for (int m = threadIdx.x; m < a.M; m += blockDim.x) {
        double c = 0.0;
        for (int k = 0; k < nk; ++k) c += a.G[(int64_t)k * a.M + m] * coef[nk + k];
        v[m] -= c;
    }
    __syncthreads();
}

// Starts the CG of one slot: r_0 = P g (the same for every realization,
// R14), lambda_0 = 0, p_0 = r_0.  A realization with r_0 = 0 is final at once.
__global__ __launch_bounds__(kThreads) void cg_init_kernel(CgArgs a) {
    __shared__ double red[kThreads / 64];
    __shared__ double coef[32];
    const int64_t l = a.init_slots[blockIdx.x];
    const int64_t q = a.slot_q[l];
    double* r = a.r + l * a.M;
    double* lam = a.lam + q * a.M;
    for (int m = threadIdx.x; m < a.M; m += blockDim.x) {
        r[m] = a.g[m];
        lam[m] = 0.0;
    }
    __syncthreads();
    if (a.nker > 0) feti_project_row(a, r, red, coef);
    double* p = a.p + l * a.M;
    double part = 0.0;
    for (int m = threadIdx.x; m < a.M; m += blockDim.x) {
        p[m] = r[m];   // p_0 = r_0
        part += r[m] * r[m];
    }
    const double rr = block_sum(part, red);
    if (threadIdx.x == 0) {
        a.rr[l] = rr;
        a.r0[l] = sqrt(rr);
        a.pend[l] = 0.0;
        a.iters[l] = 0;
        a.relres[l] = rr > 0 ? 1.0 : 0.0;
        a.status[l] = rr > 0 ? SDMM_CG_MAXITER : SDMM_CG_CONVERGED;
        a.active[l] = rr > 0 ? 1 : 0;
        if (!(rr > 0)) {
            if (a.iters_out) a.iters_out[q] = 0;
            if (a.relres_out) a.relres_out[q] = 0.0;
            if (a.status_out) a.status_out[q] = SDMM_CG_CONVERGED;
        }
    }
}

// Grouped operator: one workgroup per (subdomain i, local realization k,
// 64-row block of S_{i,k}, chunk of <= 64 realizations whose local index in
// i's KL region is k).  16-wide k-chunks of the S row block and of the
// coefficients, gathered from the global mortar layout (x: n x M) through
// i's DOF list, are staged in LDS (16.5 KB, so LDS does not limit
// occupancy); four waves compute the 64 x 64 product with FP64 MFMA
// (16x16x4, 2 x 2 tiles per wave), so each S entry is read once per chunk.  Results go
// to Y (n x sum_i R_i, subdomain-local layout) with plain stores; the CG
// update adds the two contributions of every mortar DOF in a fixed order.
typedef double dbl4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(5, 8))) void cg_apply_mfma_kernel(CgArgs a, const double* __restrict__ x,
                                                                 double* __restrict__ Y, int64_t SR,
                                                                 const int4* __restrict__ work,
                                                                 const int* __restrict__ perm) {
    constexpr int KC = 16;                       // k-chunk of S columns staged in LDS
    __shared__ double St[KC * 64];               // St[j][r] = S[row0 + r][k0 + j]
    __shared__ double Xs[KC * 65];               // Xs[j][c] = x_{l_c}[local DOF k0 + j], stride 65
    __shared__ int64_t rowoff[64];              // Y offset of each realization's block of i
    __shared__ int64_t xoff[64];                // x offset of each realization
    const int4 wk = work[blockIdx.x];   // (i, k, row0 | count << 16, perm offset)
    const int i = wk.x, k = wk.y;
    const int row0 = wk.z & 0xffff, count = wk.z >> 16;
    const int R = a.sub_R[i];
    const int nrow = min(64, R - row0);
    const double* S = a.S_cache + a.sub_Sbase[i] + (int64_t)k * R * R;
    const int64_t dptr = a.sub_dof_ptr[i];
    const int tid = threadIdx.x;
    if (tid < 64) {
        const int64_t l = tid < count ? (int64_t)perm[wk.w + tid] : -1;
        rowoff[tid] = l >= 0 ? l * SR + dptr : -1;
        xoff[tid] = l >= 0 ? l * a.M : -1;
    }
    const int64_t* dofs = a.sub_dofs + dptr;   // global mortar index of each local DOF of i
    const int lane = tid & 63, wave = tid >> 6;
    const int cb = (wave >> 1) * 32, rb = (wave & 1) * 32;   // realizations x S-rows quadrant
    const int li = lane & 15, lk = lane >> 4;
    dbl4 c00 = {0, 0, 0, 0}, c01 = c00, c10 = c00, c11 = c00;
    // Software pipeline over 16-wide k-chunks: the S and coefficient values of
    // chunk k0 + KC are loaded into registers while the MFMAs of chunk k0 run.
    // The loads are unconditional, at addresses clamped into S, the DOF list
    // and the first realization's vector, and the out-of-range values are
    // zeroed when they are staged in LDS: a masked load would need its
    // destination zeroed first, which waits for every load in flight.  Every
    // coefficient load of a thread is for local DOF k0 + (tid % KC), whose
    // global index is fetched one chunk before its coefficients.
    constexpr int NL = KC * 64 / kThreads;
    const int jt = tid % KC;
    auto dof_at = [&](int k0) { return dofs[min(k0 + jt, R - 1)]; };
    double sv[NL], xv[NL];
    auto load_chunk = [&](int k0, int64_t gj, int64_t xo0) {
#pragma unroll
        for (int q = 0; q < NL; ++q) {
            const int idx = tid + q * kThreads;
            const int j = idx >> 6, r = idx & 63;
            sv[q] = S[(int64_t)min(k0 + j, R - 1) * R + row0 + min(r, nrow - 1)];
        }
#pragma unroll
        for (int q = 0; q < NL; ++q) {
            const int64_t xo = xoff[(tid + q * kThreads) / KC];
            xv[q] = x[(xo >= 0 ? xo : xo0) + gj];
        }
    };
    int64_t gnext = dof_at(KC);
    __syncthreads();   // rowoff / xoff
    const int64_t xo0 = xoff[0];   // count >= 1
    load_chunk(0, dof_at(0), xo0);
    for (int k0 = 0; k0 < R; k0 += KC) {
        __syncthreads();   // the previous chunk's MFMAs are done with St / Xs
#pragma unroll
        for (int q = 0; q < NL; ++q) {
            const int idx = tid + q * kThreads;
            const int j = idx >> 6, r = idx & 63, c = idx / KC;
            St[idx] = (k0 + j < R && r < nrow) ? sv[q] : 0.0;
            Xs[jt * 65 + c] = (xoff[c] >= 0 && k0 + jt < R) ? xv[q] : 0.0;
        }
        __syncthreads();
        if (k0 + KC < R) {
            load_chunk(k0 + KC, gnext, xo0);
            gnext = dof_at(k0 + 2 * KC);
        }
        // transposed product Y^T = X^T S^T: tile rows are realizations, columns
        // are rows of S, so the 16 lanes of a group store 16 consecutive doubles
#pragma unroll
        for (int j0 = 0; j0 < KC; j0 += 4) {
            const double x0 = Xs[(j0 + lk) * 65 + cb + li];
            const double x1 = Xs[(j0 + lk) * 65 + cb + 16 + li];
            const double s0 = St[(j0 + lk) * 64 + rb + li];
            const double s1 = St[(j0 + lk) * 64 + rb + 16 + li];
            c00 = __builtin_amdgcn_mfma_f64_16x16x4f64(x0, s0, c00, 0, 0, 0);
            c01 = __builtin_amdgcn_mfma_f64_16x16x4f64(x0, s1, c01, 0, 0, 0);
            c10 = __builtin_amdgcn_mfma_f64_16x16x4f64(x1, s0, c10, 0, 0, 0);
            c11 = __builtin_amdgcn_mfma_f64_16x16x4f64(x1, s1, c11, 0, 0, 0);
        }
    }
    // D[i][j] (i = realization, j = S row) sits at lane j + 16 (i % 4), register i / 4
    const int jr = lane & 15, ig = lane >> 4;
    const dbl4* tiles[4] = {&c00, &c01, &c10, &c11};
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int c_base = cb + (t >> 1) * 16, r = rb + (t & 1) * 16 + jr;
        const dbl4 v = *tiles[t];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int c = c_base + 4 * q + ig;
            if (c < count && r < nrow) Y[rowoff[c] + row0 + r] = v[q];
        }
    }
}

hipError_t launch_cg_apply_mfma(const CgArgs& a, const double* x, double* Y, int64_t SR, const int4* work, int nwork,
                                const int* perm, int max_R, hipStream_t stream, hipEvent_t t0, hipEvent_t t1) {
    if (nwork <= 0) return hipSuccess;
    (void)max_R;
    if (t0 != nullptr)
        hipExtLaunchKernelGGL(cg_apply_mfma_kernel, dim3(nwork), dim3(kThreads), 0, stream, t0, t1, 0, a, x, Y, SR,
                              work, perm);
    else
        hipLaunchKernelGGL(cg_apply_mfma_kernel, dim3(nwork), dim3(kThreads), 0, stream, a, x, Y, SR, work, perm);
    return hipGetLastError();
}

// S x for the realizations of the batch into the global layout (used by the
// moments for the FETI coefficients): y_m = Y[pos1(m)] + Y[pos2(m)].
__global__ void gather_global_kernel(const double* __restrict__ Y, int64_t SR, const int* __restrict__ pos, int M,
                                     int64_t n, double* __restrict__ y) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n * M) return;
    const int64_t l = q / M;
    const int m = (int)(q - l * M);
    y[q] = Y[l * SR + pos[2 * m]] + Y[l * SR + pos[2 * m + 1]];
}

hipError_t launch_gather_global(const double* Y, int64_t SR, const int* pos, int M, int64_t n, double* y,
                                hipStream_t stream) {
    const int64_t tot = n * M;
    hipLaunchKernelGGL(gather_global_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, stream, Y, SR, pos, M,
                       n, y);
    return hipGetLastError();
}

// CG update with the operator result gathered from Y.  One workgroup per
// realization; the realization's iteration count lives in iters[l], so the
// launch is identical every iteration (graph capture).  The operator result
// is assembled in LDS (both subdomain contributions of every mortar DOF, in a
// fixed order); the FETI projection touches only the rows of G that belong to
// floating subdomains.  Two barriers per iteration without floating
// subdomains, five with; every sum has a fixed order.
// kMaxQ: vector entries per thread (M <= kThreads kMaxQ), so registers and
// LDS match the problem; W: waves per SIMD the register budget is held to
// (the most without spills: 8 up to M = 1280)
template <int kMaxQ, int W>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(W, 8))) void cg_update2_kernel(CgArgs a, const double* __restrict__ Y, int64_t SR,
                                                              const int* __restrict__ pos) {
    __shared__ double red[kThreads / 64], red2[kThreads / 64];
    __shared__ double coef[32];
    __shared__ double aps[kThreads * kMaxQ];
    const int64_t l = blockIdx.x;
    if (!a.active[l]) return;
    const int M = a.M, tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    double* r = a.r + l * M;
    double* pg = a.p + l * M;   // search direction (global layout)
    const int64_t qb = a.slot_q[l];   // the slot's realization in the batch
    double* lam = a.lam + qb * M;
    const double* Yl = Y + l * SR;
    // A p, both subdomain contributions in a fixed order; p^T A p from the
    // unprojected product (p stays in the range of the FETI projection P,
    // so p^T P A p = p^T A p)
    double pv[kMaxQ], rv[kMaxQ];
    double part = 0.0;
#pragma unroll
    for (int q = 0; q < kMaxQ; ++q) {
        const int m = tid + q * kThreads;
        pv[q] = rv[q] = 0.0;
        if (m < M) {
            const int p0 = pos[2 * m], p1 = pos[2 * m + 1];
            const double v = Yl[p0] + Yl[p1];
            aps[m] = v;
            pv[q] = pg[m];
            rv[q] = r[m];
            part += pv[q] * v;
        }
    }
    part = wave_sum(part);
    if (lane == 0) red[wid] = part;
    __syncthreads();
    const int nk = a.nker;
    if (nk > 0) {
        // c = G^T A p over the rows of floating subdomains (wave w: modes w, w + 4, ...)
        for (int kk = wid; kk < nk; kk += kThreads / 64) {
            double c = 0.0;
            for (int q = lane; q < a.nGrow; q += 64) c += a.Gval[q * nk + kk] * aps[a.Grow[q]];
            c = wave_sum(c);
            if (lane == 0) coef[kk] = c;
        }
        __syncthreads();
        if (tid < nk) {
            double d = 0.0;
            for (int q = 0; q < nk; ++q) d += a.GtGinv[tid * nk + q] * coef[q];
            coef[16 + tid] = d;
        }
        __syncthreads();
        // P A p = A p - G d on those rows
        for (int q = tid; q < a.nGrow; q += kThreads) {
            double c = 0.0;
            for (int kk = 0; kk < nk; ++kk) c += a.Gval[q * nk + kk] * coef[16 + kk];
            aps[a.Grow[q]] -= c;
        }
        __syncthreads();
    }
    double pAp = 0.0;
    for (int w = 0; w < kThreads / 64; ++w) pAp += red[w];
    const double rr = a.rr[l];
    const int iter = a.iters[l];
    // lambda update held back from the previous iteration: alpha' p' with
    // p' = (p - r) / beta' from this iteration's p = r + beta' p'
    const double pc = a.pend[l];
    if (!(pAp > 0.0) || !isfinite(pAp)) {
        if (pc != 0.0) {
#pragma unroll
            for (int q = 0; q < kMaxQ; ++q) {
                const int m = tid + q * kThreads;
                if (m < M) lam[m] += pc * (pv[q] - rv[q]);
            }
        }
        if (tid == 0) {
            a.pend[l] = 0.0;
            const double rel = a.r0[l] > 0 ? sqrt(rr) / a.r0[l] : 0.0;
            a.status[l] = SDMM_CG_BREAKDOWN;
            a.active[l] = 0;
            a.relres[l] = rel;
            if (a.iters_out) a.iters_out[qb] = iter;
            if (a.relres_out) a.relres_out[qb] = rel;
            if (a.status_out) a.status_out[qb] = SDMM_CG_BREAKDOWN;
        }
        return;
    }
    const double alpha = rr / pAp;
    // lambda moves by alpha p every iteration, but its row is read and
    // written only every other one: with a held-back update this iteration
    // adds both (the old one through p - r), otherwise it holds its own back
    // unless the realization stops here or beta is small (the held-back form
    // divides by beta; its rounding is within eps (2 / sqrt(beta) + 1) of the
    // step, as |r_new|^2 = beta |r|^2 and |p| >= |r|)
    part = 0.0;
#pragma unroll
    for (int q = 0; q < kMaxQ; ++q) {
        const int m = tid + q * kThreads;
        if (m < M) {
            const double ro = rv[q];
            rv[q] = ro - alpha * aps[m];
            if (pc != 0.0) lam[m] += pc * (pv[q] - ro) + alpha * pv[q];
            r[m] = rv[q];
        }
        part += rv[q] * rv[q];
    }
    part = wave_sum(part);
    if (lane == 0) red2[wid] = part;
    __syncthreads();
    double rrn = 0.0;
    for (int w = 0; w < kThreads / 64; ++w) rrn += red2[w];
    const double rel = sqrt(rrn) / a.r0[l];
    const bool conv = rel <= a.rtol;
    const bool last = iter + 1 >= a.max_iter;
    const double beta = rrn / rr;
    const bool hold = pc == 0.0 && !conv && !last && beta >= 1e-6;
    if (pc == 0.0 && !hold) {
#pragma unroll
        for (int q = 0; q < kMaxQ; ++q) {
            const int m = tid + q * kThreads;
            if (m < M) lam[m] += alpha * pv[q];
        }
    }
    if (tid == 0) {
        a.iters[l] = iter + 1;
        a.relres[l] = rel;
        a.pend[l] = hold ? alpha / beta : 0.0;
    }
    if (conv || last) {
        if (tid == 0) {
            const int st = conv ? SDMM_CG_CONVERGED : SDMM_CG_MAXITER;
            a.status[l] = st;
            a.active[l] = 0;
            if (a.iters_out) a.iters_out[qb] = iter + 1;
            if (a.relres_out) a.relres_out[qb] = rel;
            if (a.status_out) a.status_out[qb] = st;
        }
        return;
    }
#pragma unroll
    for (int q = 0; q < kMaxQ; ++q) {
        const int m = tid + q * kThreads;
        if (m < M) {
            pg[m] = rv[q] + beta * pv[q];
        }
    }
    if (tid == 0) a.rr[l] = rrn;
}

template <int Q>
static hipError_t launch_update2_q(const CgArgs& a, const double* Y, int64_t SR, const int* pos, hipStream_t stream,
                                   hipEvent_t t0, hipEvent_t t1) {
    auto kern = cg_update2_kernel<Q, (Q <= 3 ? 8 : Q == 4 ? 7 : Q == 5 ? 6 : Q == 6 ? 5 : 4)>;
    if (t0 != nullptr)
        hipExtLaunchKernelGGL(kern, dim3((unsigned)a.n), dim3(kThreads), 0, stream, t0, t1, 0, a, Y, SR, pos);
    else
        hipLaunchKernelGGL(kern, dim3((unsigned)a.n), dim3(kThreads), 0, stream, a, Y, SR, pos);
    return hipGetLastError();
}

hipError_t launch_cg_update2(const CgArgs& a, const double* Y, int64_t SR, const int* pos, hipStream_t stream,
                             hipEvent_t t0, hipEvent_t t1) {
    if (a.n <= 0) return hipSuccess;
    switch ((a.M + kThreads - 1) / kThreads) {
        case 0:
        case 1: return launch_update2_q<1>(a, Y, SR, pos, stream, t0, t1);
        case 2: return launch_update2_q<2>(a, Y, SR, pos, stream, t0, t1);
        case 3: return launch_update2_q<3>(a, Y, SR, pos, stream, t0, t1);
        case 4: return launch_update2_q<4>(a, Y, SR, pos, stream, t0, t1);
        case 5: return launch_update2_q<5>(a, Y, SR, pos, stream, t0, t1);
        case 6: return launch_update2_q<6>(a, Y, SR, pos, stream, t0, t1);
        case 7:
        case 8: return launch_update2_q<8>(a, Y, SR, pos, stream, t0, t1);
        default: return hipErrorInvalidValue;
    }
}

// Number of realizations of the chunk still iterating (deterministic sum).
__global__ void count_active_kernel(const int32_t* active, int64_t n, int32_t* count) {
    __shared__ int part[256];
    int s = 0;
    for (int64_t l = threadIdx.x; l < n; l += blockDim.x) s += active[l];
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int k = 0; k < (int)blockDim.x; ++k) t += part[k];
        *count = t;
    }
}

hipError_t launch_count_active(const int32_t* active, int64_t n, int32_t* count, hipStream_t stream) {
    hipLaunchKernelGGL(count_active_kernel, dim3(1), dim3(256), 0, stream, active, n, count);
    return hipGetLastError();
}

// Finished realizations of a CG stream to their callers' buffers: row
// slot[q] of lam (M values) to dst_lam[q], and its iteration count, relative
// residual and status to the optional per-realization destinations.
__global__ void stream_gather_kernel(const double* __restrict__ lam, int M, const int* __restrict__ slot,
                                     double* const* __restrict__ dst_lam, const int32_t* __restrict__ it,
                                     const double* __restrict__ rel, const int32_t* __restrict__ stat,
                                     int32_t* const* __restrict__ dst_it, double* const* __restrict__ dst_rel,
                                     int32_t* const* __restrict__ dst_st) {
    const int q = blockIdx.x;
    const int64_t l = slot[q];
    double* d = dst_lam[q];
    for (int m = threadIdx.x; m < M; m += blockDim.x) d[m] = lam[l * M + m];
    if (threadIdx.x == 0) {
        if (dst_it[q]) *dst_it[q] = it[l];
        if (dst_rel[q]) *dst_rel[q] = rel[l];
        if (dst_st[q]) *dst_st[q] = stat[l];
    }
}

hipError_t launch_stream_gather(const double* lam, int M, const int* slot, double* const* dst_lam, const int32_t* it,
                                const double* rel, const int32_t* stat, int32_t* const* dst_it,
                                double* const* dst_rel, int32_t* const* dst_st, int n, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(stream_gather_kernel, dim3(n), dim3(256), 0, stream, lam, M, slot, dst_lam, it, rel, stat,
                       dst_it, dst_rel, dst_st);
    return hipGetLastError();
}

__global__ void validate_index_kernel(const int64_t* gidx, int64_t n, int64_t nreal, int32_t* bad) {
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l < n && (gidx[l] < 0 || gidx[l] >= nreal)) *bad = 1;
}

hipError_t launch_validate_index(const int64_t* gidx, int64_t n, int64_t nreal, int32_t* bad, hipStream_t stream) {
    hipLaunchKernelGGL(validate_index_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, gidx, n, nreal,
                       bad);
    return hipGetLastError();
}

hipError_t launch_cg_init(const CgArgs& a, int64_t count, hipStream_t stream) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(cg_init_kernel, dim3((unsigned)count), dim3(kThreads), 0, stream, a);
    return hipGetLastError();
}


// ---------------------------------------------------------------------------
// Moments.  Per realization the fine fields are linear in the local mortar
// coefficients c = R_i lambda (plus the FETI kernel coefficients alpha of
// floating Stokes subdomains): u = Phi_{i,k} c + u_bar.  The accumulators
// keep, per (subdomain, local realization k), a = sum w c and
// Mc = sum w c c^T; the mean and E[u^2] of every fine DOF are then
// Phi a (+ W u_bar) and diag(Phi Mc Phi^T) (+ cross terms), the same sums
// Section 2 defines, regrouped by local realization.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void alpha_kernel(CgArgs a, const double* Slam, double* alpha) {
    __shared__ double red[kThreads / 64];
    __shared__ double coef[32];
    const int64_t l = blockIdx.x;
    const double* s = Slam + l * a.M;
    const int nk = a.nker;
    for (int k = 0; k < nk; ++k) {
        double part = 0.0;
        for (int m = threadIdx.x; m < a.M; m += blockDim.x) part += a.G[(int64_t)k * a.M + m] * (s[m] - a.g[m]);
        const double v = block_sum(part, red);
        if (threadIdx.x == 0) coef[k] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0)
        for (int k = 0; k < nk; ++k) {
            double d = 0.0;
            for (int q = 0; q < nk; ++q) d += a.GtGinv[k * nk + q] * coef[q];
            alpha[l * nk + k] = d;
        }
}

hipError_t launch_alpha(const CgArgs& a, const double* Slam, double* alpha, hipStream_t stream) {
    if (a.nker == 0) return hipSuccess;
    hipLaunchKernelGGL(alpha_kernel, dim3((unsigned)a.n), dim3(kThreads), 0, stream, a, Slam, alpha);
    return hipGetLastError();
}

// Partial moment sums of one chunk of realizations that share (i, k):
// a = sum_c w_c c and Mc = sum_c w_c c c^T over the chunk, written to the
// chunk's own slot; moments_reduce adds the slots of every (i, k) in order.
__global__ __launch_bounds__(kThreads) void accumulate_chunk_kernel(MomArgs m, const int4* __restrict__ awork,
                                                                    const int* __restrict__ perm,
                                                                    const int64_t* __restrict__ slot,
                                                                    double* __restrict__ part) {
    extern __shared__ double cs[];   // ext x 64 coefficients, then 64 weights
    const int4 wk = awork[blockIdx.x];   // (i, k, count, perm offset)
    const int i = wk.x, count = wk.z;
    const int* pl = perm + wk.w;
    const int R = m.sub_R[i], nk = m.sub_ker[i], ext = R + nk;
    const int64_t* dofs = m.sub_dofs + m.sub_dof_ptr[i];
    double* wc = cs + ext * 64;
    for (int idx = threadIdx.x; idx < ext * 64; idx += blockDim.x) {
        const int c = idx / ext, q = idx - c * ext;
        double v = 0.0;
        if (c < count) {
            const int64_t l = pl[c];
            v = q < R ? m.lam[l * m.M + dofs[q]] : m.alpha[l * m.nker + m.sub_Gcol[i] + (q - R)];
        }
        cs[q * 64 + c] = v;
    }
    for (int c = threadIdx.x; c < 64; c += blockDim.x) {
        double w = 0.0;
        if (c < count) {
            const int64_t l = pl[c];
            w = m.weights ? m.weights[l] : m.colloc_w[m.gidx[l]];
        }
        wc[c] = w;
    }
    __syncthreads();
    double* out = part + slot[blockIdx.x];
    for (int q = threadIdx.x; q < ext + ext * ext; q += blockDim.x) {
        double s = 0.0;
        if (q < ext) {
            for (int c = 0; c < count; ++c) s += wc[c] * cs[q * 64 + c];
        } else {
            const int e = q - ext, aa = e % ext, bb = e / ext;
            for (int c = 0; c < count; ++c) s += wc[c] * cs[aa * 64 + c] * cs[bb * 64 + c];
        }
        out[q] = s;
    }
}

__global__ void moments_reduce_kernel(MomArgs m, const int* __restrict__ pair_sub, const int* __restrict__ pair_k,
                                      const int* __restrict__ pair_item0, const int64_t* __restrict__ slot,
                                      const double* __restrict__ part) {
    const int pidx = blockIdx.x;
    const int i = pair_sub[pidx], k = pair_k[pidx];
    const int R = m.sub_R[i], ext = R + m.sub_ker[i];
    const int n_e = ext + ext * ext;
    double* acc = m.acc + m.sub_Abase[i] + (int64_t)k * n_e;
    const int it0 = pair_item0[pidx], it1 = pair_item0[pidx + 1];
    for (int q = blockIdx.y * blockDim.x + threadIdx.x; q < n_e; q += gridDim.y * blockDim.x) {
        double s = 0.0;
        for (int it = it0; it < it1; ++it) s += part[slot[it] + q];
        acc[q] += s;
    }
}

__global__ void lam_moments_kernel(MomArgs m) {
    const int dof = blockIdx.x * blockDim.x + threadIdx.x;
    if (dof < m.M) {
        double s1 = 0.0, s2 = 0.0;
        for (int64_t l = 0; l < m.n; ++l) {
            const double w = m.weights ? m.weights[l] : m.colloc_w[m.gidx[l]];
            const double v = m.lam[l * m.M + dof];
            s1 += w * v;
            s2 += w * v * v;
        }
        m.lam1[dof] += s1;
        m.lam2[dof] += s2;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        double ws = 0.0;
        for (int64_t l = 0; l < m.n; ++l) ws += m.weights ? m.weights[l] : m.colloc_w[m.gidx[l]];
        *m.wsum += ws;
    }
}

hipError_t launch_accumulate_chunks(const MomArgs& m, const int4* awork, int nawork, const int* perm,
                                    const int64_t* slot, double* part, const int* pair_sub, const int* pair_k,
                                    const int* pair_item0, int npairs, int max_ext, hipStream_t stream) {
    if (nawork > 0) {
        hipLaunchKernelGGL(accumulate_chunk_kernel, dim3(nawork), dim3(kThreads), (size_t)(max_ext + 1) * 64 * 8,
                           stream, m, awork, perm, slot, part);
        hipLaunchKernelGGL(moments_reduce_kernel, dim3(npairs, 16), dim3(256), 0, stream, m, pair_sub, pair_k,
                           pair_item0, slot, part);
    }
    hipLaunchKernelGGL(lam_moments_kernel, dim3((m.M + 255) / 256), dim3(256), 0, stream, m);
    return hipGetLastError();
}

// Darcy fine moments: outputs are the N cells then the RT0 edges of one
// subdomain; grid (chunk of 64 outputs, Darcy subdomain).
__device__ inline int darcy_response_row(const DarcyTables& t, const DarcyDev& D, const double* xi, const double* X,
                                         int o, double* F) {
    // fills F (R values) with the response row of output o; returns 0 when zero
    if (D.exact) return exact_response_row(t, D, xi, X, o, F);
    const int R = D.R, nx = D.nx, ny = D.ny, N = D.N;
    if (o < N) {
        const int ci = internal_of_cell(o, nx, ny, D.swap);
        for (int a = 0; a < R; ++a) F[a] = X[(int64_t)ci * R + a];
        return 1;
    }
    const int e = o - N;
    const int nv = (nx + 1) * ny;
    int c1 = -1, c2 = -1, be = -1;
    double len, hperp;
    if (e < nv) {
        const int iy = e / (nx + 1), ix = e - iy * (nx + 1);
        len = D.hy;
        hperp = D.hx;
        if (ix > 0 && ix < nx) {
            c1 = iy * nx + ix - 1;
            c2 = iy * nx + ix;
        } else {
            be = (ix == 0) ? 2 * nx + iy : 2 * nx + ny + iy;
        }
    } else {
        const int q = e - nv, iy = q / nx, ix = q - iy * nx;
        len = D.hx;
        hperp = D.hy;
        if (iy > 0 && iy < ny) {
            c1 = (iy - 1) * nx + ix;
            c2 = iy * nx + ix;
        } else {
            be = (iy == 0) ? ix : nx + ix;
        }
    }
    if (be < 0) {
        const double k1 = darcy_K(t, D, xi, c1), k2 = darcy_K(t, D, xi, c2);
        const double T = len / (D.nu * (0.5 * hperp) * (1.0 / k1 + 1.0 / k2));
        const int i1 = internal_of_cell(c1, nx, ny, D.swap), i2 = internal_of_cell(c2, nx, ny, D.swap);
        for (int a = 0; a < R; ++a) F[a] = T / len * (X[(int64_t)i1 * R + a] - X[(int64_t)i2 * R + a]);
        return 1;
    }
    const int kind = t.be_kind[D.off_be + be];
    if (kind == 2) return 0;
    const int cell = t.be_cell[D.off_be + be];
    const double kc = darcy_K(t, D, xi, cell);
    const double T = 2.0 * len * kc / (D.nu * hperp);
    const double sg = (double)t.be_sgn[D.off_be + be];
    const int ic = internal_of_cell(cell, nx, ny, D.swap);
    if (kind == 1) {
        for (int a = 0; a < R; ++a) F[a] = sg * T / len * X[(int64_t)ic * R + a];
    } else {
        const int me = t.be_medge[D.off_be + be];
        const double* Pi = t.Pi + D.off_Pi + (int64_t)me * R;
        for (int a = 0; a < R; ++a) F[a] = sg * T / len * (X[(int64_t)ic * R + a] - Pi[a]);
    }
    return 1;
}

#include "darcy_s1.inc"

__global__ __launch_bounds__(kThreads) void darcy_moments_kernel(DarcyTables t, const int* unit_of_dk, const int* d_nlocal,
                                                                 const int64_t* d_Abase, const double* acc,
                                                                 const double* X, const int64_t* cell_out_off,
                                                                 const int64_t* edge_out_off, double* p1, double* p2,
                                                                 double* u1, double* u2, int max_units_per_d) {
    extern __shared__ double F[];   // 64 outputs x R
    __shared__ double part[kThreads];
    const int d = blockIdx.y;
    const DarcyDev D = t.dar[d];
    const int R = D.R;
    const int nout = D.N + (D.nx + 1) * D.ny + D.nx * (D.ny + 1);
    const int o0 = blockIdx.x * 64;
    if (o0 >= nout) return;
    const int sub_o = threadIdx.x & 63, quarter = threadIdx.x >> 6;
    const int o = o0 + sub_o;
    double s1 = 0.0, s2 = 0.0;
    for (int k = 0; k < d_nlocal[d]; ++k) {
        const int u = unit_of_dk[d * max_units_per_d + k];
        const UnitDev U = t.units[u];
        const double* xi = t.xi + U.off_xi;
        const double* Xu = X + U.off_X;
        const double* av = acc + d_Abase[d] + (int64_t)k * (R + R * R);
        const double* Mc = av + R;
        __syncthreads();
        if (quarter == 0 && o < nout) {
            if (!darcy_response_row(t, D, xi, Xu, o, F + sub_o * R))
                for (int a = 0; a < R; ++a) F[sub_o * R + a] = 0.0;
        }
        __syncthreads();
        if (o < nout) {
            const double* f = F + sub_o * R;
            double q = 0.0, lin = 0.0;
            for (int a = quarter; a < R; a += 4) {
                double v = 0.0;
                for (int b = 0; b < R; ++b) v += Mc[(int64_t)b * R + a] * f[b];
                q += f[a] * v;
                lin += f[a] * av[a];
            }
            s1 += lin;
            s2 += q;
        }
    }
    // combine the four partial sums of every output in a fixed order
    __syncthreads();
    part[threadIdx.x] = s1;
    __syncthreads();
    double m1 = 0.0;
    if (quarter == 0) m1 = part[sub_o] + part[64 + sub_o] + part[128 + sub_o] + part[192 + sub_o];
    __syncthreads();
    part[threadIdx.x] = s2;
    __syncthreads();
    if (quarter == 0 && o < nout) {
        const double m2 = part[sub_o] + part[64 + sub_o] + part[128 + sub_o] + part[192 + sub_o];
        if (o < D.N) {
            p1[cell_out_off[d] + o] = m1;
            p2[cell_out_off[d] + o] = m2;
        } else {
            u1[edge_out_off[d] + o - D.N] = m1;
            u2[edge_out_off[d] + o - D.N] = m2;
        }
    }
}

// The same expansion with the quadratic form on FP64 MFMA (R <= 64): per
// local realization k, G = F Mc for the workgroup's 64 outputs (F: their
// response rows, 64 x R; Mc: R x R), then E[u^2] += sum_a F[o][a] G[o][a]
// and E[u] += F a.  Every thread keeps its part of the row sums across k;
// the parts are added in a fixed order at the end.
__global__ __launch_bounds__(kThreads) void darcy_moments_mfma_kernel(DarcyTables t, const int* unit_of_dk,
                                                                      const int* d_nlocal, const int64_t* d_Abase,
                                                                      const double* acc, const double* X,
                                                                      const int64_t* cell_out_off,
                                                                      const int64_t* edge_out_off, double* p1,
                                                                      double* p2, double* u1, double* u2,
                                                                      int max_units_per_d) {
    __shared__ double Fs[kTile * kLd];    // Fs[a kLd + o] = F[o][a]
    __shared__ double Ms[kTile * kLd];    // Ms[a kLd + b] = Mc[b][a]
    __shared__ double red[kTile * 33];    // row-sum parts: 16 lanes x 2 waves per row
    __shared__ double lin[kTile];
    __shared__ double Fr[kTile * kLd];    // Fr[o kLd + a] = F[o][a] as the response rows are built
    const int d = blockIdx.y;
    const DarcyDev D = t.dar[d];
    const int R = D.R;
    const int nout = D.N + (D.nx + 1) * D.ny + D.nx * (D.ny + 1);
    const int o0 = blockIdx.x * 64;
    if (o0 >= nout) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, li = lane & 15, g = lane >> 4;
    const int rb = (wave & 1) * 32, cb = (wave >> 1) * 32;
    double s2[2][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}};
    double s1 = 0.0;
    for (int k = 0; k < d_nlocal[d]; ++k) {
        const int u = unit_of_dk[d * max_units_per_d + k];
        const UnitDev U = t.units[u];
        const double* xi = t.xi + U.off_xi;
        const double* Xu = X + U.off_X;
        const double* av = acc + d_Abase[d] + (int64_t)k * (R + R * R);
        const double* Mc = av + R;
        __syncthreads();
        if (wave == 0) {
            const int o = o0 + lane;
            double* fr = Fr + lane * kLd;
            const bool has = o < nout && darcy_response_row(t, D, xi, Xu, o, fr);
            double l = 0.0;
            for (int a = 0; a < kTile; ++a) {
                if (!has || a >= R) fr[a] = 0.0;
                if (a < R) l += fr[a] * av[a];
            }
            s1 += l;
        }
        for (int idx = tid; idx < kTile * kTile; idx += kThreads) {
            const int a = idx >> 6, b = idx & 63;
            Ms[a * kLd + b] = (a < R && b < R) ? Mc[(int64_t)b * R + a] : 0.0;
        }
        __syncthreads();
        for (int idx = tid; idx < kTile * kTile; idx += kThreads) {
            const int a = idx >> 6, o = idx & 63;
            Fs[a * kLd + o] = Fr[o * kLd + a];
        }
        __syncthreads();
        TileAcc G;
        tile_acc_zero(G);
        tile_mma<false, false>(Fs, Ms, G);
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int q2 = 0; q2 < 2; ++q2)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int r = rb + 16 * p + 4 * q + g, c = cb + 16 * q2 + li;
                    s2[p][q] += G.c[p][q2][q] * Fs[c * kLd + r];
                }
    }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) red[(rb + 16 * p + 4 * q + g) * 33 + (wave >> 1) * 16 + li] = s2[p][q];
    if (wave == 0) lin[lane] = s1;
    __syncthreads();
    if (tid < 64) {
        const int o = o0 + tid;
        double m2 = 0.0;
        for (int j = 0; j < 32; ++j) m2 += red[tid * 33 + j];
        const double m1 = lin[tid];
        if (o < nout) {
            if (o < D.N) {
                p1[cell_out_off[d] + o] = m1;
                p2[cell_out_off[d] + o] = m2;
            } else {
                u1[edge_out_off[d] + o - D.N] = m1;
                u2[edge_out_off[d] + o - D.N] = m2;
            }
        }
    }
}

hipError_t launch_darcy_moments_impl(const DarcyTables& t, const int* unit_of_dk, const int* d_nlocal, int n_darcy,
                                     int max_nout, int max_units_per_d, const int64_t* d_Abase, const double* acc,
                                     const double* X, int max_R, const int64_t* cell_out_off,
                                     const int64_t* edge_out_off, double* p1, double* p2, double* u1, double* u2,
                                     hipStream_t stream) {
    if (n_darcy <= 0) return hipSuccess;
    if (max_R <= kTile)
        hipLaunchKernelGGL(darcy_moments_mfma_kernel, dim3((max_nout + 63) / 64, n_darcy), dim3(kThreads), 0, stream,
                           t, unit_of_dk, d_nlocal, d_Abase, acc, X, cell_out_off, edge_out_off, p1, p2, u1, u2,
                           max_units_per_d);
    else
        hipLaunchKernelGGL(darcy_moments_kernel, dim3((max_nout + 63) / 64, n_darcy), dim3(kThreads),
                           64 * max_R * sizeof(double), stream, t, unit_of_dk, d_nlocal, d_Abase, acc, X, cell_out_off,
                           edge_out_off, p1, p2, u1, u2, max_units_per_d);
    return hipGetLastError();
}

// Stokes fine moments: u = [U_basis, Z] c' + u_bar, p = P_basis c + p_bar.
__global__ __launch_bounds__(kThreads) void stokes_moments_kernel(const StokesDev* sd, const int64_t* s_Abase,
                                                                  const double* acc, const double* wsum,
                                                                  const double* U, const double* P, const double* Z,
                                                                  const int64_t* u_out_off, const int64_t* p_out_off,
                                                                  double* u1, double* u2, double* p1, double* p2) {
    extern __shared__ double F[];
    __shared__ double part[kThreads];
    const int si = blockIdx.y;
    const StokesDev s = sd[si];
    const int R = s.R, nk = s.nker, ext = R + nk;
    const int nout = s.nvel + s.npre;
    const int o0 = blockIdx.x * 64;
    if (o0 >= nout) return;
    const int sub_o = threadIdx.x & 63, quarter = threadIdx.x >> 6;
    const int o = o0 + sub_o;
    const double* av = acc + s_Abase[si];
    const double* Mc = av + ext;
    const double W = *wsum;
    double cbar = 0.0;
    if (quarter == 0 && o < nout) {
        double* f = F + sub_o * ext;
        if (o < s.nvel) {
            for (int a = 0; a < R; ++a) f[a] = U[s.off_U + (int64_t)a * s.nvel + o];
            for (int a = 0; a < nk; ++a) f[R + a] = Z[s.off_Z + (int64_t)a * s.nvel + o];
            cbar = U[s.off_U + (int64_t)R * s.nvel + o];
        } else {
            const int q = o - s.nvel;
            for (int a = 0; a < R; ++a) f[a] = P[s.off_P + (int64_t)a * s.npre + q];
            for (int a = 0; a < nk; ++a) f[R + a] = 0.0;
            cbar = P[s.off_P + (int64_t)R * s.npre + q];
        }
    }
    __syncthreads();
    double qv = 0.0, lin = 0.0;
    if (o < nout) {
        const double* f = F + sub_o * ext;
        for (int a = quarter; a < ext; a += 4) {
            double v = 0.0;
            for (int b = 0; b < ext; ++b) v += Mc[(int64_t)b * ext + a] * f[b];
            qv += f[a] * v;
            lin += f[a] * av[a];
        }
    }
    part[threadIdx.x] = lin;
    __syncthreads();
    double L1 = 0.0;
    if (quarter == 0) L1 = part[sub_o] + part[64 + sub_o] + part[128 + sub_o] + part[192 + sub_o];
    __syncthreads();
    part[threadIdx.x] = qv;
    __syncthreads();
    if (quarter == 0 && o < nout) {
        const double Q = part[sub_o] + part[64 + sub_o] + part[128 + sub_o] + part[192 + sub_o];
        const double m1 = L1 + W * cbar;
        const double m2 = Q + 2.0 * cbar * L1 + W * cbar * cbar;
        if (o < s.nvel) {
            u1[u_out_off[si] + o] = m1;
            u2[u_out_off[si] + o] = m2;
        } else {
            p1[p_out_off[si] + o - s.nvel] = m1;
            p2[p_out_off[si] + o - s.nvel] = m2;
        }
    }
}

hipError_t launch_stokes_moments_impl(const StokesDev* sd, int ns, int max_nout, const int64_t* s_Abase,
                                      const double* acc, const double* wsum, const double* U, const double* P,
                                      const double* Z, const int64_t* u_out_off, const int64_t* p_out_off, int max_ext,
                                      double* u1, double* u2, double* p1, double* p2, hipStream_t stream) {
    if (ns <= 0) return hipSuccess;
    hipLaunchKernelGGL(stokes_moments_kernel, dim3((max_nout + 63) / 64, ns), dim3(kThreads),
                       64 * max_ext * sizeof(double), stream, sd, s_Abase, acc, wsum, U, P, Z, u_out_off, p_out_off,
                       u1, u2, p1, p2);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Workspace of the allocation-free CG entry point (sdmm_solve_interface_
// noalloc): a fixed array in the code object, so that each GPU the library
// runs on holds its own copy from module load until the process ends.  In
// host code `scratch` names only a host-side stand-in; the device address
// of each GPU's copy comes from hipGetSymbolAddress with that GPU current,
// once per device, and every kernel argument, copy or fill uses that address.
// ---------------------------------------------------------------------------
constexpr int kScratchMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[kScratchMaxDevices] = {};
}  // namespace

hipError_t noalloc_scratch_setup(int device) {
    if (device < 0 || device >= kScratchMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return hipSuccess;
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;   // the caller makes `device` current
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = ptr;
    return hipSuccess;
}

void* noalloc_scratch_ptr(int device) {
    if (device < 0 || device >= kScratchMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_ptr[device];
}

}  // namespace sdmm
