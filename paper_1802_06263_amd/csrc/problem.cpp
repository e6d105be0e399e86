// Host-side problem setup (runs once in sdmm_set_problem).
//
// Layout and mortar maps follow Section 3.1 / 3.3 of the paper, the KL
// modes Section 2.1 with the separable kernel of eq. (covariance), the
// collocation rules Section 4 and the subdomain problems Section 5.1.  The
// orderings and readings are the ones stated in include/sdmm.h.
#include "problem.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <functional>
#include <set>

namespace sdmm {

namespace {

const double kTol = 1e-12;
const double kGx[3] = {-0.7745966692414834, 0.0, 0.7745966692414834};
const double kGw[3] = {5.0 / 9.0, 8.0 / 9.0, 5.0 / 9.0};

void mortar_shapes(int deg, double s, double* out) {
    if (deg == 1) {
        out[0] = 1.0 - s;
        out[1] = s;
    } else {
        out[0] = 2.0 * (s - 0.5) * (s - 1.0);
        out[1] = -4.0 * s * (s - 1.0);
        out[2] = 2.0 * s * (s - 0.5);
    }
}

// 1-D quadratic Lagrange shapes (nodes 0, 1/2, 1) and linear shapes on [0,1]
void q2(double s, double* v) {
    v[0] = 2.0 * (s - 0.5) * (s - 1.0);
    v[1] = -4.0 * s * (s - 1.0);
    v[2] = 2.0 * s * (s - 0.5);
}
void dq2(double s, double* v) {
    v[0] = 4.0 * s - 3.0;
    v[1] = 4.0 - 8.0 * s;
    v[2] = 4.0 * s - 1.0;
}
void q1(double s, double* v) {
    v[0] = 1.0 - s;
    v[1] = s;
}

}  // namespace

template <class G>
void Iface::node_integrals(double t0, double t1, const G& g, double* out) const {
    for (int q = 0; q < nnode; ++q) out[q] = 0.0;
    std::vector<double> cuts{t0};
    for (int e = 1; e < nelem; ++e) {
        double x = a + e * H;
        if (x > t0 + kTol && x < t1 - kTol) cuts.push_back(x);
    }
    cuts.push_back(t1);
    for (size_t k = 0; k + 1 < cuts.size(); ++k) {
        double p0 = cuts[k], p1 = cuts[k + 1];
        double mid = 0.5 * (p0 + p1), half = 0.5 * (p1 - p0);
        int e = (int)std::floor((mid - a) / H);
        e = std::min(std::max(e, 0), nelem - 1);
        for (int qp = 0; qp < 3; ++qp) {
            double t = mid + half * kGx[qp];
            double w = half * kGw[qp];
            double s = (t - (a + e * H)) / H;
            double sh[3];
            mortar_shapes(deg, s, sh);
            double gv = g(t);
            for (int n = 0; n <= deg; ++n) out[e * (deg + 1) + n] += w * gv * sh[n];
        }
    }
}

// ---------------------------------------------------------------- KL -------
// Roots of the 1-D problems for exp(-|x - x'|/eta) on [-a, a] (Section 2.1
// solved in closed form for the separable kernel of eq. covariance):
//   even modes  c cos(w a) - w sin(w a) = 0,  w a in (k pi, k pi + pi/2)
//   odd modes   w cos(w a) + c sin(w a) = 0,  w a in (k pi + pi/2, (k+1) pi)
// lambda = 2c / (w^2 + c^2), found here by plain bisection.
static void kl_1d(double a, double eta, int nmodes, std::vector<double>& lam, std::vector<double>& om,
                  std::vector<int>& par, std::vector<double>& nrm) {
    const double c = 1.0 / eta;
    const double pi = 3.14159265358979323846;
    lam.resize(nmodes);
    om.resize(nmodes);
    par.resize(nmodes);
    nrm.resize(nmodes);
    for (int n = 0; n < nmodes; ++n) {
        int k = n / 2;
        bool even = (n % 2 == 0);
        double lo = even ? k * pi / a : (k * pi + 0.5 * pi) / a;
        double hi = even ? (k * pi + 0.5 * pi) / a : (k + 1) * pi / a;
        auto f = [&](double w) {
            return even ? c * std::cos(w * a) - w * std::sin(w * a) : w * std::cos(w * a) + c * std::sin(w * a);
        };
        double flo = f(lo);
        for (int it = 0; it < 200; ++it) {
            double mid = 0.5 * (lo + hi);
            if (mid <= lo || mid >= hi) break;
            double fm = f(mid);
            if ((fm > 0) == (flo > 0)) {
                lo = mid;
                flo = fm;
            } else {
                hi = mid;
            }
        }
        double w = 0.5 * (lo + hi);
        om[n] = w;
        par[n] = even ? 0 : 1;
        lam[n] = 2.0 * c / (w * w + c * c);
        double s2 = std::sin(2.0 * w * a) / (2.0 * w);
        nrm[n] = std::sqrt(even ? a + s2 : a - s2);
    }
}

// ---------------------------------------------------------- collocation ----
// Probabilists' Gauss-Hermite nodes as the roots of He_m (recurrence
// He_{k+1} = x He_k - k He_{k-1}), bracketed on a grid and bisected; weights
// m! / (m He_{m-1}(x))^2, which sum to one for the N(0,1) density.
static void hermite(int m, double x, double& hm, double& hm1) {
    double p0 = 1.0, p1 = x;
    if (m == 0) {
        hm = 1.0;
        hm1 = 0.0;
        return;
    }
    for (int k = 1; k < m; ++k) {
        double p2 = x * p1 - k * p0;
        p0 = p1;
        p1 = p2;
    }
    hm = p1;
    hm1 = p0;
}

static void gauss_hermite(int m, std::vector<double>& x, std::vector<double>& w) {
    x.clear();
    w.clear();
    if (m == 1) {
        x.push_back(0.0);
        w.push_back(1.0);
        return;
    }
    double R = std::sqrt(4.0 * m + 6.0) + 1.0;
    int steps = 400 * m;
    double prev_x = -R, hm, hm1;
    hermite(m, prev_x, hm, hm1);
    double prev_v = hm;
    for (int s = 1; s <= steps; ++s) {
        double xx = -R + 2.0 * R * s / steps;
        hermite(m, xx, hm, hm1);
        if (hm == 0.0 || (hm > 0) != (prev_v > 0)) {
            double lo = prev_x, hi = xx, flo = prev_v;
            for (int it = 0; it < 200; ++it) {
                double mid = 0.5 * (lo + hi);
                if (mid <= lo || mid >= hi) break;
                double fm, d;
                hermite(m, mid, fm, d);
                if ((fm > 0) == (flo > 0)) {
                    lo = mid;
                    flo = fm;
                } else {
                    hi = mid;
                }
            }
            x.push_back(0.5 * (lo + hi));
        }
        prev_x = xx;
        prev_v = hm;
    }
    // symmetry of the rule
    for (int i = 0; i < m / 2; ++i) {
        double v = 0.5 * (x[m - 1 - i] - x[i]);
        x[i] = -v;
        x[m - 1 - i] = v;
    }
    if (m % 2 == 1) x[m / 2] = 0.0;
    double fact = 1.0;
    for (int k = 2; k <= m; ++k) fact *= k;
    double tot = 0.0;
    for (int i = 0; i < m; ++i) {
        hermite(m, x[i], hm, hm1);
        double wi = fact / ((double)m * m * hm1 * hm1);
        w.push_back(wi);
        tot += wi;
    }
    for (int i = 0; i < m; ++i) w[i] /= tot;
    for (int i = 0; i < m / 2; ++i) {
        double v = 0.5 * (w[i] + w[m - 1 - i]);
        w[i] = w[m - 1 - i] = v;
    }
}

static double binom(int n, int k) {
    if (k < 0 || k > n) return 0.0;
    double r = 1.0;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return std::round(r);
}

// ------------------------------------------------------------ layout -------
static bool shared_segment(const Sub& s, const Sub& t, int& horizontal, double& coord, double& a, double& b) {
    const double ya[2][2] = {{s.y1, t.y0}, {s.y0, t.y1}};
    for (auto& pr : ya) {
        if (std::fabs(pr[0] - pr[1]) < kTol) {
            a = std::max(s.x0, t.x0);
            b = std::min(s.x1, t.x1);
            if (b - a > kTol) {
                horizontal = 1;
                coord = pr[0];
                return true;
            }
        }
    }
    const double xa[2][2] = {{s.x1, t.x0}, {s.x0, t.x1}};
    for (auto& pr : xa) {
        if (std::fabs(pr[0] - pr[1]) < kTol) {
            a = std::max(s.y0, t.y0);
            b = std::min(s.y1, t.y1);
            if (b - a > kTol) {
                horizontal = 0;
                coord = pr[0];
                return true;
            }
        }
    }
    return false;
}

// side: 0 bottom, 1 top, 2 left, 3 right
static int iface_at(const Problem& P, int i, int side, double t) {
    const Sub& s = P.subs[i];
    int hor = side < 2;
    double c = side == 0 ? s.y0 : side == 1 ? s.y1 : side == 2 ? s.x0 : s.x1;
    for (int fi : P.sub_ifaces[i]) {
        const Iface& f = P.ifaces[fi];
        if (f.horizontal == hor && std::fabs(f.coord - c) < kTol && t >= f.a - kTol && t <= f.b + kTol) return fi;
    }
    return -1;
}

static int local_offset(const Problem& P, int i, int fi) {
    for (size_t k = 0; k < P.sub_ifaces[i].size(); ++k)
        if (P.sub_ifaces[i][k] == fi) return P.sub_dof_off[i][k];
    return -1;
}

// --------------------------------------------------------- Darcy ----------
static std::string build_darcy(Problem& P, int i, DarcyHost& d) {
    const Sub& s = P.subs[i];
    d.sub = i;
    d.nx = s.nx;
    d.ny = s.ny;
    d.N = s.nx * s.ny;
    d.swap = s.nx > s.ny ? 1 : 0;
    d.b = std::min(s.nx, s.ny);
    d.exact = P.in.darcy_mass == 1;
    d.Ns = d.exact ? std::max(s.nx, s.ny) * (2 * d.b + 1) + d.b : d.N;
    d.bs = d.exact ? 2 * d.b + 1 : d.b;
    d.hx = s.hx;
    d.hy = s.hy;
    d.R = (int)(P.sub_ptr[i + 1] - P.sub_ptr[i]);
    d.n_medge = 0;
    struct Pending { int medge; int fi; double t0, t1, len; };
    std::vector<Pending> pend;
    for (int side = 0; side < 4; ++side) {
        int nedge = side < 2 ? s.nx : s.ny;
        double h = side < 2 ? s.hx : s.hy;
        double hperp = side < 2 ? s.hy : s.hx;
        double base = side < 2 ? s.x0 : s.y0;
        for (int k = 0; k < nedge; ++k) {
            double t0 = base + k * h, t1 = base + (k + 1) * h;
            int cell, edge;
            int nv = (s.nx + 1) * s.ny;
            if (side == 0) { cell = k; edge = nv + k; }
            else if (side == 1) { cell = (s.ny - 1) * s.nx + k; edge = nv + s.ny * s.nx + k; }
            else if (side == 2) { cell = k * s.nx; edge = k * (s.nx + 1); }
            else { cell = k * s.nx + s.nx - 1; edge = k * (s.nx + 1) + s.nx; }
            int fi = iface_at(P, i, side, 0.5 * (t0 + t1));
            int kind;
            if (fi >= 0) kind = 0;
            else if (side == 0 && std::fabs(s.y0 - P.in.domain[2]) < kTol) kind = 1;
            else kind = 2;
            d.be_cell.push_back(cell);
            d.be_kind.push_back(kind);
            d.be_len.push_back(h);
            d.be_hperp.push_back(hperp);
            d.be_sgn.push_back((side == 0 || side == 2) ? -1 : 1);
            d.be_edge.push_back(edge);
            if (kind == 0) {
                d.be_medge.push_back(d.n_medge);
                pend.push_back({d.n_medge, fi, t0, t1, h});
                d.n_medge++;
            } else {
                d.be_medge.push_back(-1);
            }
        }
    }
    d.Pi.assign((size_t)d.n_medge * d.R, 0.0);
    std::vector<double> tmp(64);
    for (auto& pe : pend) {
        const Iface& f = P.ifaces[pe.fi];
        f.node_integrals(pe.t0, pe.t1, [](double) { return 1.0; }, tmp.data());
        int off = local_offset(P, i, pe.fi);
        for (int q = 0; q < f.nnode; ++q) d.Pi[(size_t)pe.medge * d.R + off + q] = tmp[q] / pe.len;
    }
    // mortar functions must not outnumber the fine edges they act on
    for (int fi : P.sub_ifaces[i]) {
        const Iface& f = P.ifaces[fi];
        int nfine = (int)std::lround((f.b - f.a) / (f.horizontal ? s.hx : s.hy));
        if (f.nnode > nfine) return "a mortar has more degrees of freedom than the fine trace of a Darcy subdomain";
    }
    // KL: the terms of the region (their values at the cell centres are
    // computed on the device)
    d.nterm = P.region_nterm[s.region];
    d.mean_logk = P.region_mean[s.region];
    return "";
}

// --------------------------------------------------------- Stokes ---------
// Symmetric 3x3 eigen-decomposition by cyclic Jacobi rotations.
static void jacobi3(double A[3][3], double V[3][3], double ev[3]) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) V[i][j] = (i == j);
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = std::fabs(A[0][1]) + std::fabs(A[0][2]) + std::fabs(A[1][2]);
        if (off < 1e-300) break;
        for (int p = 0; p < 2; ++p)
            for (int q = p + 1; q < 3; ++q) {
                if (std::fabs(A[p][q]) < 1e-300) continue;
                double th = 0.5 * (A[q][q] - A[p][p]) / A[p][q];
                double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
                double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < 3; ++k) {
                    double akp = A[k][p], akq = A[k][q];
                    A[k][p] = c * akp - s * akq;
                    A[k][q] = s * akp + c * akq;
                }
                for (int k = 0; k < 3; ++k) {
                    double apk = A[p][k], aqk = A[q][k];
                    A[p][k] = c * apk - s * aqk;
                    A[q][k] = s * apk + c * aqk;
                }
                for (int k = 0; k < 3; ++k) {
                    double vkp = V[k][p], vkq = V[k][q];
                    V[k][p] = c * vkp - s * vkq;
                    V[k][q] = s * vkp + c * vkq;
                }
            }
    }
    for (int i = 0; i < 3; ++i) ev[i] = A[i][i];
}

struct Trip { int r, c; double v; };

static void compress(std::vector<Trip>& t) {
    std::sort(t.begin(), t.end(), [](const Trip& a, const Trip& b) { return a.r != b.r ? a.r < b.r : a.c < b.c; });
    size_t w = 0;
    for (size_t k = 0; k < t.size(); ++k) {
        if (w > 0 && t[w - 1].r == t[k].r && t[w - 1].c == t[k].c) t[w - 1].v += t[k].v;
        else t[w++] = t[k];
    }
    t.resize(w);
}

// P2-P1 (triangular Taylor-Hood, the pair of the numerical cases of Section
// 6) on one rectangle cut into two right triangles, accumulated into the
// 18x18 / 4x18 blocks of the Q2-Q1 layout: the P2 nodes of both triangles are
// the 3x3 node grid of the rectangle (node 3b+a at (a hx/2, b hy/2), the
// diagonal midpoint is the centre) and the P1 pressures its four corners.
// cut 0 runs the diagonal from (0,0) to (hx,hy), cut 1 from (hx,0) to (0,hy).
// With barycentric coordinates l_k every P2 gradient is linear,
//   grad(l_i (2 l_i - 1)) = sum_k (4 delta_ik - 1) l_k grad l_i,
//   grad(4 l_i l_j)       = 4 l_j grad l_i + 4 l_i grad l_j,
// so both forms are sums of the exact moments int_T l_k l_l = |T| (1 + delta_kl) / 12.
static void p2p1_blocks(double hx, double hy, double nu, int cut, double Ae[18][18], double Be[4][18]) {
    static const int tri[2][2][3][2] = {{{{0, 0}, {2, 0}, {2, 2}}, {{0, 0}, {2, 2}, {0, 2}}},
                                        {{{0, 0}, {2, 0}, {0, 2}}, {{2, 0}, {2, 2}, {0, 2}}}};
    for (int m = 0; m < 18; ++m) {
        for (int n = 0; n < 18; ++n) Ae[m][n] = 0.0;
        for (int q = 0; q < 4; ++q) Be[q][m] = 0.0;
    }
    for (int t = 0; t < 2; ++t) {
        const int(*v)[2] = tri[cut][t];
        double x[3], y[3];
        for (int k = 0; k < 3; ++k) {
            x[k] = 0.5 * hx * v[k][0];
            y[k] = 0.5 * hy * v[k][1];
        }
        const double det = (x[1] - x[0]) * (y[2] - y[0]) - (x[2] - x[0]) * (y[1] - y[0]);
        const double area = 0.5 * std::fabs(det);
        double gl[3][2];  // grad l_k
        for (int k = 0; k < 3; ++k) {
            const int a = (k + 1) % 3, b = (k + 2) % 3;
            gl[k][0] = (y[a] - y[b]) / det;
            gl[k][1] = (x[b] - x[a]) / det;
        }
        // six P2 functions: node on the 3x3 grid, gradient coefficients c[k] (grad = sum_k l_k c[k])
        int node[6];
        double c[6][3][2] = {};
        for (int i = 0; i < 3; ++i) {
            node[i] = 3 * v[i][1] + v[i][0];
            for (int k = 0; k < 3; ++k)
                for (int d = 0; d < 2; ++d) c[i][k][d] = (k == i ? 3.0 : -1.0) * gl[i][d];
        }
        for (int e = 0; e < 3; ++e) {
            const int i = e, j = (e + 1) % 3;
            node[3 + e] = 3 * ((v[i][1] + v[j][1]) / 2) + (v[i][0] + v[j][0]) / 2;
            for (int d = 0; d < 2; ++d) {
                c[3 + e][j][d] = 4.0 * gl[i][d];
                c[3 + e][i][d] = 4.0 * gl[j][d];
            }
        }
        int pn[3];
        for (int k = 0; k < 3; ++k) pn[k] = 2 * (v[k][1] / 2) + v[k][0] / 2;
        double mom[3][3];
        for (int k = 0; k < 3; ++k)
            for (int l = 0; l < 3; ++l) mom[k][l] = area * (k == l ? 2.0 : 1.0) / 12.0;
        for (int m = 0; m < 6; ++m)
            for (int n = 0; n < 6; ++n) {
                double g[2][2] = {};  // g[dm][dn] = int d_dm(phi_m) d_dn(phi_n)
                for (int k = 0; k < 3; ++k)
                    for (int l = 0; l < 3; ++l)
                        for (int dm = 0; dm < 2; ++dm)
                            for (int dn = 0; dn < 2; ++dn) g[dm][dn] += c[m][k][dm] * c[n][l][dn] * mom[k][l];
                const int M = node[m], N = node[n];
                Ae[2 * M][2 * N] += nu * (2.0 * g[0][0] + g[1][1]);
                Ae[2 * M + 1][2 * N + 1] += nu * (2.0 * g[1][1] + g[0][0]);
                Ae[2 * M + 1][2 * N] += nu * g[0][1];
                Ae[2 * M][2 * N + 1] += nu * g[1][0];
            }
        for (int n = 0; n < 6; ++n)
            for (int q = 0; q < 3; ++q)
                for (int d = 0; d < 2; ++d) {
                    double s = 0.0;
                    for (int k = 0; k < 3; ++k) s += c[n][k][d] * mom[k][q];
                    Be[pn[q]][2 * node[n] + d] -= s;
                }
    }
}

static std::string build_stokes(Problem& P, int i, StokesHost& S) {
    const Sub& s = P.subs[i];
    const sdmm_problem& in = P.in;
    S.sub = i;
    S.nx = s.nx;
    S.ny = s.ny;
    const int nnx = 2 * s.nx + 1, nny = 2 * s.ny + 1;
    S.nvel = 2 * nnx * nny;
    S.npre = (s.nx + 1) * (s.ny + 1);
    S.R = (int)(P.sub_ptr[i + 1] - P.sub_ptr[i]);
    const double nu = in.nu_s;
    // 1-D integrals on [0,1] by 3-point Gauss (exact for these degrees)
    double M2[3][3] = {}, K2[3][3] = {}, D2[3][3] = {}, ML[3][2] = {}, DL[3][2] = {};
    for (int g = 0; g < 3; ++g) {
        double t = 0.5 * (1.0 + kGx[g]), w = 0.5 * kGw[g];
        double v[3], dv[3], l[2];
        q2(t, v);
        dq2(t, dv);
        q1(t, l);
        for (int a = 0; a < 3; ++a) {
            for (int b = 0; b < 3; ++b) {
                M2[a][b] += w * v[a] * v[b];
                K2[a][b] += w * dv[a] * dv[b];
                D2[a][b] += w * dv[a] * v[b];
            }
            for (int q = 0; q < 2; ++q) {
                ML[a][q] += w * v[a] * l[q];
                DL[a][q] += w * dv[a] * l[q];
            }
        }
    }
    const double hx = s.hx, hy = s.hy;
    // element blocks from tensor products of the 1-D integrals
    double Ae[18][18] = {}, Be[4][18] = {};
    for (int bm = 0; bm < 3; ++bm)
        for (int am = 0; am < 3; ++am)
            for (int bn = 0; bn < 3; ++bn)
                for (int an = 0; an < 3; ++an) {
                    int m = 3 * bm + am, n = 3 * bn + an;
                    double xx = (hy / hx) * K2[an][am] * M2[bn][bm];
                    double yy = (hx / hy) * M2[an][am] * K2[bn][bm];
                    // int d_y(phi_n) d_x(phi_m) and its transpose partner
                    double yx = D2[am][an] * D2[bn][bm];
                    double xy = D2[an][am] * D2[bm][bn];
                    Ae[2 * m][2 * n] += nu * (2.0 * xx + yy);
                    Ae[2 * m + 1][2 * n + 1] += nu * (2.0 * yy + xx);
                    Ae[2 * m + 1][2 * n] += nu * yx;
                    Ae[2 * m][2 * n + 1] += nu * xy;
                }
    for (int qb = 0; qb < 2; ++qb)
        for (int qa = 0; qa < 2; ++qa)
            for (int bn = 0; bn < 3; ++bn)
                for (int an = 0; an < 3; ++an) {
                    int q = 2 * qb + qa, n = 3 * bn + an;
                    Be[q][2 * n] -= hy * DL[an][qa] * ML[bn][qb];
                    Be[q][2 * n + 1] -= hx * ML[an][qa] * DL[bn][qb];
                }
    // the triangular pair: two cuts (the lower-right and upper-left corner
    // rectangles take the diagonal through their outer corner, so no triangle
    // has two edges on the subdomain boundary)
    double At[2][18][18], Bt[2][4][18];
    const bool tri = in.stokes_element == 1;
    if (tri)
        for (int c = 0; c < 2; ++c) p2p1_blocks(hx, hy, nu, c, At[c], Bt[c]);
    std::vector<Trip> A, B;
    A.reserve((size_t)s.nx * s.ny * 324 + 1000);
    B.reserve((size_t)s.nx * s.ny * 72);
    for (int ey = 0; ey < s.ny; ++ey)
        for (int ex = 0; ex < s.nx; ++ex) {
            int dofs[18], pn[4];
            for (int b = 0; b < 3; ++b)
                for (int a = 0; a < 3; ++a) {
                    int node = (2 * ey + b) * nnx + 2 * ex + a;
                    dofs[2 * (3 * b + a)] = 2 * node;
                    dofs[2 * (3 * b + a) + 1] = 2 * node + 1;
                }
            for (int b = 0; b < 2; ++b)
                for (int a = 0; a < 2; ++a) pn[2 * b + a] = (ey + b) * (s.nx + 1) + ex + a;
            const int cut = (ex == s.nx - 1 && ey == 0) || (ex == 0 && ey == s.ny - 1);
            const double(*Ause)[18] = tri ? At[cut] : Ae;
            const double(*Buse)[18] = tri ? Bt[cut] : Be;
            for (int m = 0; m < 18; ++m)
                for (int n = 0; n < 18; ++n)
                    if (Ause[m][n] != 0.0) A.push_back({dofs[m], dofs[n], Ause[m][n]});
            for (int q = 0; q < 4; ++q)
                for (int n = 0; n < 18; ++n)
                    if (Buse[q][n] != 0.0) B.push_back({pn[q], dofs[n], Buse[q][n]});
        }
    // boundary: Dirichlet nodes, traces against mortar functions, BJS
    std::vector<char> dir(nnx * nny, 0);
    std::vector<std::vector<std::pair<int, double>>> Qrows(S.R);
    const double bjs = nu * in.alpha / std::sqrt(in.k_bjs);
    std::vector<double> tmp(64);
    for (int side = 0; side < 4; ++side) {
        int nel = side < 2 ? s.nx : s.ny;
        double h = side < 2 ? hx : hy;
        double base = side < 2 ? s.x0 : s.y0;
        double nrm[2] = {side == 2 ? -1.0 : side == 3 ? 1.0 : 0.0, side == 0 ? -1.0 : side == 1 ? 1.0 : 0.0};
        int tang = side < 2 ? 0 : 1;
        for (int e = 0; e < nel; ++e) {
            int nodes[3];
            for (int k = 0; k < 3; ++k) {
                int p = 2 * e + k;
                if (side == 0) nodes[k] = p;
                else if (side == 1) nodes[k] = (nny - 1) * nnx + p;
                else if (side == 2) nodes[k] = p * nnx;
                else nodes[k] = p * nnx + nnx - 1;
            }
            double t0 = base + e * h, t1 = t0 + h;
            int fi = iface_at(P, i, side, 0.5 * (t0 + t1));
            if (fi < 0) {
                for (int k = 0; k < 3; ++k) dir[nodes[k]] = 1;
                continue;
            }
            const Iface& f = P.ifaces[fi];
            int off = local_offset(P, i, fi);
            for (int k = 0; k < 3; ++k) {
                f.node_integrals(t0, t1, [&](double t) { double v[3]; q2((t - t0) / h, v); return v[k]; }, tmp.data());
                for (int nd = 0; nd < f.nnode; ++nd) {
                    if (tmp[nd] == 0.0) continue;
                    if (f.kind == 0) {
                        for (int c = 0; c < 2; ++c) {
                            int q = off + 2 * nd + c;
                            double sg = (double)P.sub_sign[P.sub_ptr[i] + q];
                            Qrows[q].push_back({2 * nodes[k] + c, sg * tmp[nd]});
                        }
                    } else {
                        int q = off + nd;
                        for (int c = 0; c < 2; ++c)
                            if (nrm[c] != 0.0) Qrows[q].push_back({2 * nodes[k] + c, nrm[c] * tmp[nd]});
                    }
                }
            }
            if (f.kind == 1) {
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b)
                        A.push_back({2 * nodes[a] + tang, 2 * nodes[b] + tang, bjs * h * M2[a][b]});
            }
        }
    }
    compress(A);
    compress(B);
    int nd_dir = 0;
    for (char c : dir) nd_dir += c;
    S.floating = nd_dir == 0;
    S.uD.assign(S.nvel, 0.0);
    // imposed outer velocity (inflow_x + inflow_shear y, inflow_y)
    for (int n = 0; n < nnx * nny; ++n)
        if (dir[n]) {
            const double yn = s.y0 + 0.5 * hy * (n / nnx);
            S.uD[2 * n] = in.inflow_x + in.inflow_shear * yn;
            S.uD[2 * n + 1] = in.inflow_y;
        }
    // kernel of the velocity form for floating subdomains
    std::vector<char> pinned(S.nvel, 0);
    S.nker = 0;
    std::vector<double> Zraw;
    if (S.floating) {
        double xc = 0.5 * (s.x0 + s.x1), yc = 0.5 * (s.y0 + s.y1);
        std::vector<double> rig((size_t)S.nvel * 3, 0.0);
        for (int iy = 0; iy < nny; ++iy)
            for (int ix = 0; ix < nnx; ++ix) {
                int n = iy * nnx + ix;
                double x = s.x0 + 0.5 * ix * hx, y = s.y0 + 0.5 * iy * hy;
                rig[(size_t)(2 * n) * 3 + 0] = 1.0;
                rig[(size_t)(2 * n + 1) * 3 + 1] = 1.0;
                rig[(size_t)(2 * n) * 3 + 2] = -(y - yc);
                rig[(size_t)(2 * n + 1) * 3 + 2] = x - xc;
            }
        double G[3][3] = {};
        for (const Trip& t : A)
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) G[a][b] += rig[(size_t)t.r * 3 + a] * t.v * rig[(size_t)t.c * 3 + b];
        double V[3][3], ev[3];
        jacobi3(G, V, ev);
        double emax = std::max(1.0, std::max(std::fabs(ev[0]), std::max(std::fabs(ev[1]), std::fabs(ev[2]))));
        std::vector<int> keep;
        for (int k = 0; k < 3; ++k)
            if (ev[k] < 1e-10 * emax) keep.push_back(k);
        S.nker = (int)keep.size();
        Zraw.assign((size_t)S.nvel * S.nker, 0.0);
        for (int c = 0; c < S.nker; ++c)
            for (int r = 0; r < S.nvel; ++r) {
                double v = 0;
                for (int a = 0; a < 3; ++a) v += rig[(size_t)r * 3 + a] * V[a][keep[c]];
                Zraw[(size_t)c * S.nvel + r] = v;
            }
        // modified Gram-Schmidt: orthonormal columns
        for (int c = 0; c < S.nker; ++c) {
            for (int c2 = 0; c2 < c; ++c2) {
                double dot = 0;
                for (int r = 0; r < S.nvel; ++r) dot += Zraw[(size_t)c * S.nvel + r] * Zraw[(size_t)c2 * S.nvel + r];
                for (int r = 0; r < S.nvel; ++r) Zraw[(size_t)c * S.nvel + r] -= dot * Zraw[(size_t)c2 * S.nvel + r];
            }
            double nn = 0;
            for (int r = 0; r < S.nvel; ++r) nn += Zraw[(size_t)c * S.nvel + r] * Zraw[(size_t)c * S.nvel + r];
            nn = std::sqrt(nn);
            for (int r = 0; r < S.nvel; ++r) Zraw[(size_t)c * S.nvel + r] /= nn;
        }
        // pin one velocity DOF per kernel vector (elimination with row pivoting)
        std::vector<double> W = Zraw;
        for (int c = 0; c < S.nker; ++c) {
            int best = -1;
            double bv = 0;
            for (int r = 0; r < S.nvel; ++r)
                if (!pinned[r] && std::fabs(W[(size_t)c * S.nvel + r]) > bv) {
                    bv = std::fabs(W[(size_t)c * S.nvel + r]);
                    best = r;
                }
            pinned[best] = 1;
            for (int c2 = c + 1; c2 < S.nker; ++c2) {
                double f = W[(size_t)c2 * S.nvel + best] / W[(size_t)c * S.nvel + best];
                for (int r = 0; r < S.nvel; ++r) W[(size_t)c2 * S.nvel + r] -= f * W[(size_t)c * S.nvel + r];
            }
        }
        P.n_kernel += S.nker;
    }
    // band ordering: nodes row-major, free velocity DOFs of each node; the
    // pressures of the vertices of an element follow its centre node
    std::vector<int> vband(S.nvel, -1), pband(S.npre, -1);
    std::vector<std::vector<int>> pres_after(nnx * nny);
    for (int b = 0; b <= s.ny; ++b)
        for (int a = 0; a <= s.nx; ++a) {
            int ex = std::min(a, s.nx - 1), ey = std::min(b, s.ny - 1);
            pres_after[(2 * ey + 1) * nnx + 2 * ex + 1].push_back(b * (s.nx + 1) + a);
        }
    int nb = 0;
    for (int n = 0; n < nnx * nny; ++n) {
        for (int c = 0; c < 2; ++c) {
            int d = 2 * n + c;
            if (!dir[n] && !pinned[d]) {
                vband[d] = nb++;
                S.band_kind.push_back(0);
                S.band_raw.push_back(d);
            }
        }
        for (int pq : pres_after[n]) {
            pband[pq] = nb++;
            S.band_kind.push_back(1);
            S.band_raw.push_back(pq);
        }
    }
    S.nband = nb;
    S.bw = 0;
    for (const Trip& t : A) {
        int r = vband[t.r], c = vband[t.c];
        if (r < 0 || c < 0 || r < c) continue;
        S.ar.push_back(r);
        S.ac.push_back(c);
        S.av.push_back(t.v);
        S.bw = std::max(S.bw, r - c);
    }
    for (const Trip& t : B) {
        int pr = pband[t.r], vc = vband[t.c];
        if (vc < 0) continue;
        int r = std::max(pr, vc), c = std::min(pr, vc);
        S.ar.push_back(r);
        S.ac.push_back(c);
        S.av.push_back(t.v);
        S.bw = std::max(S.bw, r - c);
    }
    // right-hand sides: R basis loads -Q^T e_j (compatible part for floating
    // subdomains) and the complementary load from the Dirichlet data
    const int nc = S.R + 1;
    S.rhs.assign((size_t)nb * nc, 0.0);
    std::vector<double> f(S.nvel);
    for (int j = 0; j < S.R; ++j) {
        std::fill(f.begin(), f.end(), 0.0);
        for (auto& pr : Qrows[j]) f[pr.first] -= pr.second;
        for (int c = 0; c < S.nker; ++c) {
            double dot = 0;
            for (int r = 0; r < S.nvel; ++r) dot += Zraw[(size_t)c * S.nvel + r] * f[r];
            for (int r = 0; r < S.nvel; ++r) f[r] -= dot * Zraw[(size_t)c * S.nvel + r];
        }
        for (int r = 0; r < S.nvel; ++r)
            if (vband[r] >= 0) S.rhs[(size_t)j * nb + vband[r]] = f[r];
    }
    for (const Trip& t : A)
        if (vband[t.r] >= 0 && dir[t.c / 2]) S.rhs[(size_t)S.R * nb + vband[t.r]] -= t.v * S.uD[t.c];
    for (const Trip& t : B)
        if (dir[t.c / 2]) S.rhs[(size_t)S.R * nb + pband[t.r]] -= t.v * S.uD[t.c];
    // trace rows over raw velocity DOFs
    S.q_ptr.assign(S.R + 1, 0);
    for (int j = 0; j < S.R; ++j) {
        std::map<int, double> row;
        for (auto& pr : Qrows[j]) row[pr.first] += pr.second;
        for (auto& kv : row) {
            S.q_col.push_back(kv.first);
            S.q_val.push_back(kv.second);
        }
        S.q_ptr[j + 1] = (int)S.q_col.size();
    }
    S.Z = Zraw;  // nker x nvel, column c contiguous
    return "";
}

// ------------------------------------------------------------ driver ------
std::string build_problem(const sdmm_problem& in, Problem& P) {
    P = Problem();
    P.in = in;
    if (in.n_sub <= 0 || !in.sub_type || !in.sub_rect || !in.sub_n || !in.sub_region) return "no subdomains";
    if (in.mortar_degree != 1 && in.mortar_degree != 2) return "mortar degree must be 1 or 2";
    if (in.stokes_element != 0 && in.stokes_element != 1) return "Stokes element must be 0 (Q2-Q1) or 1 (P2-P1)";
    if (in.darcy_mass != 0 && in.darcy_mass != 1) return "Darcy mass must be 0 (trapezoidal) or 1 (exact)";
    if (in.mortar_elements < 1) return "mortar elements must be positive";
    if (in.p_bottom != 0.0) return "the GPU path requires p_bottom == 0";
    if (in.nu_s <= 0 || in.nu_d <= 0 || in.k_bjs <= 0 || in.alpha < 0) return "invalid physical parameters";
    for (int i = 0; i < in.n_sub; ++i) {
        Sub s;
        s.type = in.sub_type[i];
        s.x0 = in.sub_rect[4 * i];
        s.x1 = in.sub_rect[4 * i + 1];
        s.y0 = in.sub_rect[4 * i + 2];
        s.y1 = in.sub_rect[4 * i + 3];
        s.nx = in.sub_n[2 * i];
        s.ny = in.sub_n[2 * i + 1];
        s.region = in.sub_region[i];
        if (s.type != 0 && s.type != 1) return "subdomain type must be 0 (Stokes) or 1 (Darcy)";
        if (s.nx < 1 || s.ny < 1 || !(s.x1 > s.x0) || !(s.y1 > s.y0)) return "invalid subdomain mesh";
        s.hx = (s.x1 - s.x0) / s.nx;
        s.hy = (s.y1 - s.y0) / s.ny;
        if (s.type == 0) {
            if (!P.subs.empty() && P.subs.back().type == 1) return "Stokes subdomains must come first";
            P.n_stokes++;
        } else {
            P.n_darcy++;
            if (s.region < 0 || s.region >= in.n_region) return "Darcy subdomain with an invalid KL region";
            // every cell has at most two boundary faces; the face-pressure band
            // (2 min(nx, ny) + 1) is factored in the LDS window up to 55 cells and
            // as 64 x 64 tiles in device memory above (kept to 128 cells)
            if (in.darcy_mass == 1 && (std::min(s.nx, s.ny) < 2 || std::min(s.nx, s.ny) > 128))
                return "the exact RT0 mass needs 2 <= min(nx, ny) <= 128 on every Darcy subdomain";
        }
        P.subs.push_back(s);
    }
    // tiling check: subdomain areas sum to the domain area, no overlaps
    double area = 0;
    for (auto& s : P.subs) area += (s.x1 - s.x0) * (s.y1 - s.y0);
    double darea = (in.domain[1] - in.domain[0]) * (in.domain[3] - in.domain[2]);
    if (std::fabs(area - darea) > 1e-9 * darea) return "subdomains do not tile the domain";
    for (size_t a = 0; a < P.subs.size(); ++a)
        for (size_t b = a + 1; b < P.subs.size(); ++b) {
            const Sub &s = P.subs[a], &t = P.subs[b];
            double ox = std::min(s.x1, t.x1) - std::max(s.x0, t.x0);
            double oy = std::min(s.y1, t.y1) - std::max(s.y0, t.y0);
            if (ox > kTol && oy > kTol) return "subdomains overlap";
        }
    // interfaces
    const int nsub = in.n_sub;
    P.sub_ifaces.assign(nsub, {});
    int off = 0;
    for (int i = 0; i < nsub; ++i)
        for (int j = i + 1; j < nsub; ++j) {
            Iface f;
            if (!shared_segment(P.subs[i], P.subs[j], f.horizontal, f.coord, f.a, f.b)) continue;
            f.i = i;
            f.j = j;
            int ti = P.subs[i].type, tj = P.subs[j].type;
            f.kind = (ti == 0 && tj == 0) ? 0 : (ti == 1 && tj == 1) ? 2 : 1;
            f.ncomp = f.kind == 0 ? 2 : 1;
            f.nelem = in.mortar_elements;
            f.deg = in.mortar_degree;
            f.nnode = f.nelem * (f.deg + 1);
            f.ndof = f.nnode * f.ncomp;
            f.H = (f.b - f.a) / f.nelem;
            f.off = off;
            off += f.ndof;
            P.sub_ifaces[i].push_back((int)P.ifaces.size());
            P.sub_ifaces[j].push_back((int)P.ifaces.size());
            P.ifaces.push_back(f);
        }
    P.M = off;
    P.sub_ptr.assign(nsub + 1, 0);
    P.sub_dof_off.assign(nsub, {});
    for (int i = 0; i < nsub; ++i) {
        int loc = 0;
        for (int fi : P.sub_ifaces[i]) {
            const Iface& f = P.ifaces[fi];
            P.sub_dof_off[i].push_back(loc);
            int sg = (f.kind == 0 && f.j == i) ? -1 : 1;
            for (int q = 0; q < f.ndof; ++q) {
                P.sub_dofs.push_back(f.off + q);
                P.sub_sign.push_back(sg);
            }
            loc += f.ndof;
        }
        P.sub_ptr[i + 1] = P.sub_ptr[i] + loc;
    }
    // KL regions
    P.n_region = in.n_region;
    if (P.n_region < 1) return "at least one KL region is needed";
    P.nterm = 0;
    P.dim_off.push_back(0);
    for (int r = 0; r < P.n_region; ++r) {
        for (int k = 0; k < 4; ++k) P.region_rect.push_back(in.region_rect[4 * r + k]);
        int nt = in.region_nterm[r];
        if (nt < 0) return "negative number of KL terms";
        P.region_nterm.push_back(nt);
        P.region_sigma2.push_back(in.region_sigma2[r]);
        P.region_eta.push_back(in.region_eta[2 * r]);
        P.region_eta.push_back(in.region_eta[2 * r + 1]);
        P.region_mean.push_back(in.region_mean_logk[r]);
        if (!(in.region_eta[2 * r] > 0) || !(in.region_eta[2 * r + 1] > 0) || in.region_sigma2[r] < 0)
            return "invalid KL parameters";
        P.nterm += nt;
        P.dim_off.push_back(P.nterm);
        KLRegion K;
        double x0 = in.region_rect[4 * r], x1 = in.region_rect[4 * r + 1];
        double y0 = in.region_rect[4 * r + 2], y1 = in.region_rect[4 * r + 3];
        K.xc = 0.5 * (x0 + x1);
        K.yc = 0.5 * (y0 + y1);
        int nm = nt + 1;
        std::vector<double> lx, ly;
        kl_1d(0.5 * (x1 - x0), in.region_eta[2 * r], nm, lx, K.wx, K.px, K.nx_);
        kl_1d(0.5 * (y1 - y0), in.region_eta[2 * r + 1], nm, ly, K.wy, K.py, K.ny_);
        struct Cand { double neg; int s, a, b; };
        std::vector<Cand> cand;
        for (int a = 0; a < nm; ++a)
            for (int b = 0; b < nm; ++b) cand.push_back({-(in.region_sigma2[r] * lx[a] * ly[b]), a + b, a, b});
        std::sort(cand.begin(), cand.end(), [](const Cand& u, const Cand& v) {
            if (u.neg != v.neg) return u.neg < v.neg;
            if (u.s != v.s) return u.s < v.s;
            return u.a < v.a;
        });
        for (int t = 0; t < nt; ++t) {
            K.ma.push_back(cand[t].a);
            K.mb.push_back(cand[t].b);
            K.lam.push_back(-cand[t].neg);
        }
        P.kl.push_back(K);
    }
    for (int i = 0; i < nsub; ++i) {
        const Sub& s = P.subs[i];
        if (s.type != 1) continue;
        const double* rr = &in.region_rect[4 * s.region];
        if (s.x0 < rr[0] - kTol || s.x1 > rr[1] + kTol || s.y0 < rr[2] - kTol || s.y1 > rr[3] + kTol)
            return "a KL region is not a union of its Darcy subdomains";
    }
    // collocation
    const int N = P.nterm;
    if (in.rule_kind == 0) {
        int m = in.rule_m;
        if (m < 1) return "tensor rule needs m >= 1";
        double tot = std::pow((double)m, N);
        if (tot > 5e6) return "tensor grid too large";
        std::vector<double> x, w;
        gauss_hermite(m, x, w);
        P.node_x = x;
        P.nreal = (int64_t)std::llround(tot);
        P.ids.assign((size_t)P.nreal * N, 0);
        P.weights.assign(P.nreal, 1.0);
        for (int64_t l = 0; l < P.nreal; ++l) {
            int64_t rem = l;
            for (int d = N - 1; d >= 0; --d) {
                int dig = (int)(rem % m);
                rem /= m;
                P.ids[(size_t)l * N + d] = dig;
                P.weights[l] *= w[dig];
            }
        }
    } else if (in.rule_kind == 1) {
        int L = in.rule_level;
        if (L < 0 || L > 6) return "sparse level must be in 0..6";
        std::vector<std::vector<double>> rx(L + 1), rw(L + 1);
        std::vector<double> all;
        for (int p = 0; p <= L; ++p) {
            int m = in.rule_growth == 0 ? (1 << (p + 1)) - 1 : p + 1;
            gauss_hermite(m, rx[p], rw[p]);
            for (double v : rx[p]) all.push_back(v);
        }
        std::sort(all.begin(), all.end());
        std::vector<double> uniq;
        for (double v : all)
            if (uniq.empty() || std::fabs(v - uniq.back()) > 1e-10) uniq.push_back(v);
        bool has0 = false;
        for (double v : uniq) has0 |= std::fabs(v) < 1e-13;
        if (has0) P.node_x.push_back(0.0);
        for (double v : uniq)
            if (std::fabs(v) >= 1e-13) P.node_x.push_back(v);
        auto nid = [&](double v) {
            int best = 0;
            for (size_t k = 1; k < P.node_x.size(); ++k)
                if (std::fabs(P.node_x[k] - v) < std::fabs(P.node_x[best] - v)) best = (int)k;
            return best;
        };
        std::vector<std::vector<int>> rid(L + 1);
        for (int p = 0; p <= L; ++p)
            for (double v : rx[p]) rid[p].push_back(nid(v));
        std::map<std::vector<uint8_t>, double> acc;
        int lmin = std::max(0, L - N + 1);
        std::vector<int> comp(N, 0);
        std::function<void(int, int)> rec = [&](int d, int left) {
            if (d == N - 1) {
                comp[d] = left;
                int tot = 0;
                for (int v : comp) tot += v;
                double coef = ((L - tot) % 2 ? -1.0 : 1.0) * binom(N - 1, L - tot);
                // tensor product of the 1-D rules
                std::vector<int> idx(N, 0);
                std::vector<uint8_t> key(N);
                while (true) {
                    double wv = coef;
                    for (int k = 0; k < N; ++k) {
                        key[k] = (uint8_t)rid[comp[k]][idx[k]];
                        wv *= rw[comp[k]][idx[k]];
                    }
                    acc[key] += wv;
                    int k = N - 1;
                    while (k >= 0) {
                        if (++idx[k] < (int)rx[comp[k]].size()) break;
                        idx[k] = 0;
                        --k;
                    }
                    if (k < 0) break;
                }
                return;
            }
            for (int v = 0; v <= left; ++v) {
                comp[d] = v;
                rec(d + 1, left - v);
            }
        };
        if (N == 0) {
            P.nreal = 1;
            P.weights.assign(1, 1.0);
        } else {
            for (int tot = lmin; tot <= L; ++tot) rec(0, tot);
            P.nreal = (int64_t)acc.size();
            P.ids.reserve((size_t)P.nreal * N);
            for (auto& kv : acc) {
                for (int k = 0; k < N; ++k) P.ids.push_back(kv.first[k]);
                P.weights.push_back(kv.second);
            }
        }
    } else {
        return "rule kind must be 0 (tensor) or 1 (sparse)";
    }
    // local sets and the global -> local table
    P.g2l.assign((size_t)P.nreal * P.n_region, 0);
    for (int r = 0; r < P.n_region; ++r) {
        int o = P.dim_off[r], nt = P.region_nterm[r];
        std::map<std::vector<int32_t>, int> loc;
        for (int64_t l = 0; l < P.nreal; ++l)
            loc.emplace(std::vector<int32_t>(P.ids.begin() + l * N + o, P.ids.begin() + l * N + o + nt), 0);
        int k = 0;
        std::vector<int32_t> flat;
        for (auto& kv : loc) {
            kv.second = k++;
            flat.insert(flat.end(), kv.first.begin(), kv.first.end());
        }
        P.local_ids.push_back(flat);
        P.nlocal.push_back(k);
        for (int64_t l = 0; l < P.nreal; ++l)
            P.g2l[(size_t)l * P.n_region + r] =
                loc[std::vector<int32_t>(P.ids.begin() + l * N + o, P.ids.begin() + l * N + o + nt)];
    }
    // subdomain operators
    for (int i = 0; i < nsub; ++i) {
        if (P.subs[i].type == 1) {
            DarcyHost d;
            std::string err = build_darcy(P, i, d);
            if (!err.empty()) return err;
            P.darcy.push_back(std::move(d));
        } else {
            StokesHost s;
            std::string err = build_stokes(P, i, s);
            if (!err.empty()) return err;
            P.stokes.push_back(std::move(s));
        }
    }
    return "";
}

}  // namespace sdmm
