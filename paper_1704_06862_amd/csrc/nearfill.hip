// FP64 near-field fill on the device: the same matrix as fill_near
// (nearfield.cpp) - PMCHWT blocks, or the JMCFIE / CNF blocks with their
// normal-field integrals and Gram terms - one thread per stored edge pair.
//
// A thread owns entry (row m, column n) of a finest box's row-major block
// and sums, over the sides (triangle P of m, triangle Q of n) and the regions
// r that border both, the (i, j) element of the local interactions of P and
// Q (i, j: the local indices of m in P and of n in Q).  Each thread writes its
// own entry, so the result does not depend on scheduling.  The work per pair
// of triangles is repeated for each of the up to nine entries it feeds; the
// fill is bound by the FP64 Green's-function evaluations, not by memory.
//
// Integrals (eqs. 3-9, exp(+j w t), G = exp(-jkR)/(4 pi R)), as on the host:
// 7-point outer and inner rules; for a pair that shares a vertex or whose
// centroids are closer than twice the longer of their longest edges, the
// terms (1/R - k^2 R/2)/(4 pi) and their gradient are integrated over Q in
// closed form (edge integrals of R^-1, R, R^3 and the solid angle) and the
// rule integrates only the remainder.  K of a triangle with itself is 0.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <vector>

#include "core.hpp"
#include "device.hpp"
#include "fp64dev.hpp"

namespace sfmm {

namespace {

using namespace fp64;

#define NFCHK(x)                                                                                      \
    do {                                                                                              \
        hipError_t e_ = (x);                                                                          \
        if (e_ != hipSuccess) throw Error(SFMM_E_DEVICE, std::string("near fill: ") + hipGetErrorString(e_)); \
    } while (0)

// per-triangle geometry, structure of arrays
struct TriGeo {
    const double *v;      // [nt][3 vertices][3]
    const double *n;      // [nt][3] unit normal
    const double *c;      // [nt][3] centroid
    const double *qp;     // [nt][7][3] quadrature nodes
    const double *area, *maxedge;
    const int *vid;       // [nt][3] vertex ids
    const int *tr;        // [nt][2] (front region, back region)
    const int *tsign;     // [nt][3] coefficient of the half basis of local vertex i
};

struct EdgeSides {
    const int *nside;     // [ne]
    const int *tri;       // [ne][3]
    const int *loc;       // [ne][3] local index of the edge in that triangle
    const double *len;    // [ne]
};

struct FillArgs {
    TriGeo g;
    EdgeSides e;
    const zc *k, *eta;    // per region
    double w[7];          // 7-point rule weights (sum 1)
    int nb;
    const int64_t *val_ptr;
    const int *col_ptr, *cols, *bstart, *order;
    int gen, tang;        // general blocks (JMCFIE / CNF); T parts present (JMCFIE)
    zc *A, *B, *C, *D;
};

__device__ inline d3 ld3(const double *p) { return {p[0], p[1], p[2]}; }

__device__ inline int region_sign(const TriGeo &g, int t, int r) {
    return g.tr[2 * t] == r ? 1 : (g.tr[2 * t + 1] == r ? -1 : 0);
}

// ln((R+ + s+)/(R- + s-)) through the equal form with the larger arguments
__device__ inline double edge_log(double rp, double sp, double rm, double sm) {
    const double n1 = rp + sp, d1 = rm + sm, n2 = rm - sm, d2 = rp - sp;
    const double v = (fmin(n1, d1) >= fmin(n2, d2)) ? log(n1 / d1) : log(n2 / d2);
    return isfinite(v) ? v : 0.0;
}

struct Closed {
    double inv_r, r1;
    d3 v_inv_r, v_r1, g_inv_r, g_r1, rho;
};

// Int_Q 1/R, R, (rho' - rho)/R, (rho' - rho) R, grad 1/R, grad R at point r
__device__ Closed closed_form(d3 r, const d3 *p, d3 n, bool in_plane) {
    Closed c;
    const double h = in_plane ? 0.0 : dotp(r - p[0], n);
    const double ah = fabs(h);
    c.rho = r - h * n;
    double sum_te_m1 = 0, sum_te1 = 0, sum_beta = 0;
    d3 sm_e1{0, 0, 0}, sm_e3{0, 0, 0}, sm_em1{0, 0, 0};
    for (int i = 0; i < 3; ++i) {
        const d3 a = p[i], b = p[(i + 1) % 3];
        d3 s = b - a;
        s = (1.0 / normp(s)) * s;
        const d3 mh = crossp(s, n);
        const double s_lo = dotp(a - c.rho, s), s_hi = dotp(b - c.rho, s);
        const double t = dotp(a - c.rho, mh);
        const double r0sq = t * t + h * h;
        const double R_lo = normp(r - a), R_hi = normp(r - b);
        const double e_m1 = edge_log(R_hi, s_hi, R_lo, s_lo);
        const double e_1 = 0.5 * (s_hi * R_hi - s_lo * R_lo + r0sq * e_m1);
        const double e_3 = 0.25 * (s_hi * R_hi * R_hi * R_hi - s_lo * R_lo * R_lo * R_lo + 3.0 * r0sq * e_1);
        double beta = 0.0;
        if (r0sq + ah * fmin(R_hi, R_lo) > 0)
            beta = atan2(t * s_hi, r0sq + ah * R_hi) - atan2(t * s_lo, r0sq + ah * R_lo);
        sum_te_m1 += t * e_m1;
        sum_te1 += t * e_1;
        sum_beta += beta;
        sm_e1 = sm_e1 + e_1 * mh;
        sm_e3 = sm_e3 + e_3 * mh;
        sm_em1 = sm_em1 + e_m1 * mh;
    }
    c.inv_r = sum_te_m1 - ah * sum_beta;
    c.r1 = (sum_te1 + h * h * c.inv_r) / 3.0;
    const double sg = h > 0 ? 1.0 : (h < 0 ? -1.0 : 0.0);
    c.v_inv_r = sm_e1;
    c.v_r1 = (1.0 / 3.0) * sm_e3;
    c.g_inv_r = (-1.0) * sm_em1 - (sg * sum_beta) * n;
    c.g_r1 = (-1.0) * sm_e1 + (h * c.inv_r) * n;
    return c;
}

__device__ inline zc expmj(zc k, double R) {   // exp(-j k R)
    const double mag = exp(k.i * R);
    double sn, cs;
    sincos(k.r * R, &sn, &cs);
    return {mag * cs, -mag * sn};
}

__device__ inline bool close_pair(const TriGeo &g, int P, int Q) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            if (g.vid[3 * P + i] == g.vid[3 * Q + j]) return true;
    const d3 d = ld3(g.c + 3 * P) - ld3(g.c + 3 * Q);
    return normp(d) < 2.0 * fmax(g.maxedge[P], g.maxedge[Q]);
}

// Element (i, j) of the local interactions of test triangle P and source
// triangle Q for the wavenumbers of regions r0 (and r1 if nr == 2): L, K and,
// with normal testing, LN, KN (fields tested with n_P x h_i).
struct Local {
    zc L, K, LN, KN;
};

__device__ void pair_element(const FillArgs &a, int P, int Q, int i, int j, const int *regs, int nr, bool close,
                             bool ntest, Local *out) {
    const TriGeo &g = a.g;
    const double AP = g.area[P], AQ = g.area[Q];
    const bool same = P == Q;
    const d3 pi_ = ld3(g.v + 9 * P + 3 * i);
    const d3 qj = ld3(g.v + 9 * Q + 3 * j);
    const d3 np = ld3(g.n + 3 * P);
    d3 qv[3];
    for (int u = 0; u < 3; ++u) qv[u] = ld3(g.v + 9 * Q + 3 * u);
    const d3 nq = ld3(g.n + 3 * Q);
    const double inv4pi = 0.25 / M_PI;
    zc Lacc[2] = {{0, 0}, {0, 0}}, Kacc[2] = {{0, 0}, {0, 0}}, LNacc[2] = {{0, 0}, {0, 0}},
       KNacc[2] = {{0, 0}, {0, 0}};
    for (int ia = 0; ia < 7; ++ia) {
        const d3 ra = ld3(g.qp + 21 * P + 3 * ia);
        Closed cf;
        if (close) cf = closed_form(ra, qv, nq, same);
        const d3 ri = ra - pi_, rj = ra - qj;
        const d3 ti = crossp(np, ri);
        const double wa = a.w[ia] * AP;
        for (int s = 0; s < nr; ++s) {
            const zc k = a.k[regs[s]];
            zc Isc{0, 0};
            zv Iv{{0, 0}, {0, 0}, {0, 0}}, gg{{0, 0}, {0, 0}, {0, 0}};
            for (int ib = 0; ib < 7; ++ib) {
                const d3 rb = ld3(g.qp + 21 * Q + 3 * ib);
                const d3 d = ra - rb;
                const double R = normp(d);
                const double wb = a.w[ib] * AQ;
                zc G, gf;
                if (close) {
                    if (R > 0) {
                        const zc e = expmj(k, R);
                        const zc kr = R * k;
                        const zc half = 0.5 * (kr * kr);
                        G = (inv4pi / R) * (e - zc{1, 0} + half);
                        // -(1 + j kR) e + 1 + (kR)^2 / 2
                        const zc jkr{-kr.i, kr.r};
                        gf = (inv4pi / (R * R * R)) * (zc{1, 0} + half - (zc{1, 0} + jkr) * e);
                    } else {
                        G = inv4pi * zc{k.i, -k.r};   // -j k / (4 pi)
                        gf = {0, 0};
                    }
                } else {
                    const zc e = expmj(k, R);
                    G = (inv4pi / R) * e;
                    const zc jkr{-k.i * R, k.r * R};
                    gf = (-inv4pi / (R * R * R)) * ((zc{1, 0} + jkr) * e);
                }
                const zc wG = wb * G, wg = wb * gf;
                Isc = Isc + wG;
                Iv.x = Iv.x + rb.x * wG;
                Iv.y = Iv.y + rb.y * wG;
                Iv.z = Iv.z + rb.z * wG;
                gg.x = gg.x + d.x * wg;
                gg.y = gg.y + d.y * wg;
                gg.z = gg.z + d.z * wg;
            }
            if (close) {
                const zc k2h = 0.5 * (k * k);
                const zc ssc = inv4pi * (zc{cf.inv_r, 0} - cf.r1 * k2h);
                Isc = Isc + ssc;
                Iv.x = Iv.x + inv4pi * (zc{cf.v_inv_r.x, 0} - cf.v_r1.x * k2h) + cf.rho.x * ssc;
                Iv.y = Iv.y + inv4pi * (zc{cf.v_inv_r.y, 0} - cf.v_r1.y * k2h) + cf.rho.y * ssc;
                Iv.z = Iv.z + inv4pi * (zc{cf.v_inv_r.z, 0} - cf.v_r1.z * k2h) + cf.rho.z * ssc;
                gg.x = gg.x + inv4pi * (zc{cf.g_inv_r.x, 0} - cf.g_r1.x * k2h);
                gg.y = gg.y + inv4pi * (zc{cf.g_inv_r.y, 0} - cf.g_r1.y * k2h);
                gg.z = gg.z + inv4pi * (zc{cf.g_inv_r.z, 0} - cf.g_r1.z * k2h);
            }
            // vec = Ivec - q_j Isc; L: (r - p_i).vec - (4 / k^2) Isc
            zv vec{Iv.x - qj.x * Isc, Iv.y - qj.y * Isc, Iv.z - qj.z * Isc};
            const zc four_k2 = zdiv(zc{4, 0}, k * k);
            Lacc[s] = Lacc[s] + wa * (zdot(ri, vec) - four_k2 * Isc);
            // K: (r - p_i).(g x (r - q_j)); complex g times real vector
            zv cr{gg.y * rj.z - gg.z * rj.y, gg.z * rj.x - gg.x * rj.z, gg.x * rj.y - gg.y * rj.x};
            Kacc[s] = Kacc[s] + wa * zdot(ri, cr);
            if (ntest) {
                // A_Q L h_j = (-j k / 2)(Ivec - q_j Isc) - (j / k) g
                const zc mjk2{0.5 * k.i, -0.5 * k.r};         // -j k / 2
                const zc mjok = zdiv(zc{0, -1}, k);             // -j / k
                zv lh{mjk2 * vec.x + mjok * gg.x, mjk2 * vec.y + mjok * gg.y, mjk2 * vec.z + mjok * gg.z};
                LNacc[s] = LNacc[s] + wa * zdot(ti, lh);
                KNacc[s] = KNacc[s] + wa * zdot(ti, cr);
            }
        }
    }
    for (int s = 0; s < nr; ++s) {
        const zc k = a.k[regs[s]];
        const zc lf = (1.0 / (4.0 * AP * AQ)) * zc{k.i, -k.r};   // -j k / (4 A_P A_Q)
        out[s].L = lf * Lacc[s];
        out[s].K = same ? zc{0, 0} : (1.0 / (4.0 * AP * AQ)) * Kacc[s];
        if (ntest) {
            out[s].LN = (1.0 / (2.0 * AP * AQ)) * LNacc[s];
            out[s].KN = same ? zc{0, 0} : (1.0 / (4.0 * AP * AQ)) * KNacc[s];
        }
    }
}

// Gram elements of triangle P's half bases: int_P h_i . h_j, int_P h_i . (n x h_j)
__device__ void gram_element(const FillArgs &a, int P, int i, int j, double &G, double &GN) {
    const TriGeo &g = a.g;
    const double A = g.area[P];
    const d3 pi_ = ld3(g.v + 9 * P + 3 * i), pj = ld3(g.v + 9 * P + 3 * j), n = ld3(g.n + 3 * P);
    G = GN = 0;
    for (int ia = 0; ia < 7; ++ia) {
        const double w = a.w[ia] * A / (4.0 * A * A);
        const d3 r = ld3(g.qp + 21 * P + 3 * ia);
        const d3 hi = r - pi_, hj = r - pj;
        G += w * dotp(hi, hj);
        GN += w * dotp(hi, crossp(n, hj));
    }
}

__global__ void __launch_bounds__(128) k_near_fill(const FillArgs a) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nnz = a.val_ptr[a.nb];
    if (id >= nnz) return;
    // box of this entry: the last b with val_ptr[b] <= id
    int lo = 0, hi = a.nb - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a.val_ptr[mid] <= id) lo = mid;
        else hi = mid - 1;
    }
    const int b = lo;
    const int ncol = a.col_ptr[b + 1] - a.col_ptr[b];
    const int64_t off = id - a.val_ptr[b];
    const int row = (int)(off / ncol), col = (int)(off % ncol);
    const int m = a.order[a.bstart[b] + row];
    const int n = a.order[a.cols[a.col_ptr[b] + col]];
    const TriGeo &g = a.g;
    const double ts = -1.0;   // weight of the T parts in JMCFIE
    zc A{0, 0}, B{0, 0}, C{0, 0}, D{0, 0};
    for (int si = 0; si < a.e.nside[m]; ++si) {
        const int P = a.e.tri[3 * m + si], li = a.e.loc[3 * m + si];
        const double smu = g.tsign[3 * P + li] * a.e.len[m];
        for (int sj = 0; sj < a.e.nside[n]; ++sj) {
            const int Q = a.e.tri[3 * n + sj], lj = a.e.loc[3 * n + sj];
            const double snu = g.tsign[3 * Q + lj] * a.e.len[n];
            int regs[2], nr = 0;
            for (int rr = 0; rr < 2; ++rr) {
                const int r = g.tr[2 * P + rr];
                if (g.tr[2 * Q] == r || g.tr[2 * Q + 1] == r) regs[nr++] = r;
            }
            if (nr) {
                Local loc[2];
                pair_element(a, P, Q, li, lj, regs, nr, close_pair(g, P, Q), a.gen != 0, loc);
                for (int s = 0; s < nr; ++s) {
                    const int r = regs[s];
                    const zc et = a.eta[r];
                    const double f = region_sign(g, P, r) * region_sign(g, Q, r) * smu * snu;
                    if (!a.gen) {
                        A = A + f * (et * loc[s].L);
                        B = B + f * loc[s].K;
                        C = C + f * zdiv(loc[s].L, et);
                        continue;
                    }
                    const double fn = region_sign(g, Q, r) * smu * snu;
                    zc av = fn * loc[s].KN, bv = (-fn) * zdiv(loc[s].LN, et), dv = (-fn) * (et * loc[s].LN);
                    if (a.tang) {
                        av = av + (ts * f) * loc[s].L;
                        bv = bv + (ts * f) * zdiv(loc[s].K, et);
                        dv = dv + (ts * f) * (et * loc[s].K);
                    }
                    A = A + av;
                    B = B + bv;
                    C = C + av;
                    D = D + dv;
                }
            }
            if (a.gen && P == Q) {
                double Gm, GN;
                gram_element(a, P, li, lj, Gm, GN);
                const zc eo = a.eta[g.tr[2 * P]], ep = a.eta[g.tr[2 * P + 1]];
                zc wj{0, 0}, wm{0, 0};
                if (a.tang) {
                    wj = (0.5 * ts) * (eo - ep);
                    wm = (-0.5 * ts) * (zdiv(zc{1, 0}, eo) - zdiv(zc{1, 0}, ep));
                }
                const double f = smu * snu;
                A = A + zc{f * Gm, 0};
                C = C + zc{f * Gm, 0};
                B = B - (f * GN) * wm;
                D = D + (f * GN) * wj;
            }
        }
    }
    a.A[id] = A;
    a.B[id] = B;
    a.C[id] = C;
    if (a.gen) a.D[id] = D;
}

template <typename U>
U *dup(const std::vector<U> &v, std::vector<void *> &owned) {
    U *p = nullptr;
    NFCHK(hipMalloc(&p, sizeof(U) * std::max<size_t>(v.size(), 1)));
    owned.push_back(p);
    if (!v.empty()) NFCHK(hipMemcpy(p, v.data(), sizeof(U) * v.size(), hipMemcpyHostToDevice));
    return p;
}

}  // namespace

NearMatrix fill_near_device(const Mesh &m, const Octree &o, int form, int device) {
    NearMatrix Z = near_structure(o);
    const int64_t nnz = Z.val_ptr[o.nb];
    const bool gen = form != SFMM_FORM_PMCHWT;
    Z.A.assign(nnz, 0.0);
    Z.B.assign(nnz, 0.0);
    Z.C.assign(nnz, 0.0);
    if (gen) Z.D.assign(nnz, 0.0);
    if (nnz == 0) return Z;
    NFCHK(hipSetDevice(device));
    std::vector<double> v((size_t)9 * m.nt), nrm((size_t)3 * m.nt), cen((size_t)3 * m.nt), qp((size_t)21 * m.nt);
    std::vector<int> vid((size_t)3 * m.nt), tr((size_t)2 * m.nt), ts((size_t)3 * m.nt);
    for (int t = 0; t < m.nt; ++t) {
        for (int u = 0; u < 3; ++u) {
            for (int c = 0; c < 3; ++c) v[9 * t + 3 * u + c] = m.V[m.T[t][u]][c];
            vid[3 * t + u] = m.T[t][u];
            ts[3 * t + u] = m.tri_sign[t][u];
            nrm[3 * t + u] = m.normal[t][u];
            cen[3 * t + u] = m.centroid[t][u];
        }
        for (int q = 0; q < 7; ++q)
            for (int c = 0; c < 3; ++c) qp[21 * t + 3 * q + c] = m.qp[t][q][c];
        tr[2 * t] = m.TR[t][0];
        tr[2 * t + 1] = m.TR[t][1];
    }
    std::vector<int> nside(m.ne), etri((size_t)3 * m.ne, -1), eloc((size_t)3 * m.ne, -1);
    for (int e = 0; e < m.ne; ++e) {
        nside[e] = m.nside[e];
        for (int i = 0; i < m.nside[e]; ++i) {
            const int t = m.etri[e][i];
            etri[3 * e + i] = t;
            for (int l = 0; l < 3; ++l)
                if (m.tri_edge[t][l] == e) eloc[3 * e + i] = l;
            if (eloc[3 * e + i] < 0) throw Error(SFMM_E_MESH, "edge missing from its triangle");
        }
    }
    std::vector<double> kk((size_t)2 * m.nr), ee((size_t)2 * m.nr);
    for (int r = 0; r < m.nr; ++r) {
        kk[2 * r] = m.k[r].real();
        kk[2 * r + 1] = m.k[r].imag();
        ee[2 * r] = m.eta[r].real();
        ee[2 * r + 1] = m.eta[r].imag();
    }
    std::vector<void *> owned;
    auto release = [&] {
        for (void *p : owned) (void)hipFree(p);
        owned.clear();
    };
    try {
        FillArgs a{};
        a.g.v = dup(v, owned);
        a.g.n = dup(nrm, owned);
        a.g.c = dup(cen, owned);
        a.g.qp = dup(qp, owned);
        a.g.area = dup(m.area, owned);
        a.g.maxedge = dup(m.maxedge, owned);
        a.g.vid = dup(vid, owned);
        a.g.tr = dup(tr, owned);
        a.g.tsign = dup(ts, owned);
        a.e.nside = dup(nside, owned);
        a.e.tri = dup(etri, owned);
        a.e.loc = dup(eloc, owned);
        a.e.len = dup(m.len, owned);
        a.k = reinterpret_cast<const zc *>(dup(kk, owned));
        a.eta = reinterpret_cast<const zc *>(dup(ee, owned));
        const TriRule &q = tri_rule();
        for (int i = 0; i < 7; ++i) a.w[i] = q.w[i];
        a.nb = o.nb;
        a.val_ptr = dup(Z.val_ptr, owned);
        a.col_ptr = dup(Z.col_ptr, owned);
        a.cols = dup(Z.cols, owned);
        a.bstart = dup(o.bstart, owned);
        a.order = dup(o.order, owned);
        a.gen = gen;
        a.tang = form != SFMM_FORM_CNF;
        zc *planes[4] = {nullptr, nullptr, nullptr, nullptr};
        for (int p = 0; p < (gen ? 4 : 3); ++p) {
            NFCHK(hipMalloc(&planes[p], sizeof(zc) * nnz));
            owned.push_back(planes[p]);
        }
        a.A = planes[0];
        a.B = planes[1];
        a.C = planes[2];
        a.D = planes[3];
        const int bs = 128;
        const int64_t nblk = (nnz + bs - 1) / bs;
        hipLaunchKernelGGL(k_near_fill, dim3((unsigned)nblk), dim3(bs), 0, 0, a);
        NFCHK(hipGetLastError());
        NFCHK(hipDeviceSynchronize());
        std::vector<cd> *dst[4] = {&Z.A, &Z.B, &Z.C, &Z.D};
        for (int p = 0; p < (gen ? 4 : 3); ++p)
            NFCHK(hipMemcpy(dst[p]->data(), planes[p], sizeof(zc) * nnz, hipMemcpyDeviceToHost));
    } catch (...) {
        release();
        throw;
    }
    release();
    return Z;
}

}  // namespace sfmm
