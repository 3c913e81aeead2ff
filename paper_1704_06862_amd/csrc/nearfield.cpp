// FP64 near-field matrix of the scaled PMCHWT system.
//
// Operators (eqs. 3-7 of the paper, exp(+j w t), G = exp(-jkR)/(4 pi R)):
//   L[m,n] = -jk  Int Int [ f_m . f_n - k^-2 div f_m div' f_n ] G
//   K[m,n] =      Int Int   f_m(r) . ( grad G(r, r') x f_n(r') )      (principal value)
// and the PMCHWT block of an edge pair summed over the regions r that border
// both edges, with region signs s (eqs. 10-13, 16):
//   A = sum s s et_r L_r,   B = sum s s K_r,   C = sum s s L_r / et_r,
//   block = [[A, -B], [B, C]] acting on (J, M~ = M/eta0), E-rows divided by eta0.
//
// Integration: the 7-point rule for outer and inner integrals.  For triangle
// pairs that share a vertex or whose centroids are closer than twice the
// longer of their longest edges, (1/R - k^2 R/2)/(4 pi) and its gradient are
// integrated over the source triangle in closed form (Wilton et al. 1984,
// Graglia 1993: edge integrals of R^-1, R, R^3 and the solid-angle term) and
// the rule integrates only the smooth remainder.  K of a triangle with itself
// vanishes (all vectors lie in one plane) and is not computed.
//
// Because grad G is parallel to r - r', grad G x (r' - v) = grad G x (r - v),
// so the K inner integral needs only Int grad G dS'.
#include <algorithm>
#include <cmath>
#include <omp.h>

#include "core.hpp"

namespace sfmm {

namespace {

struct Closed {
    double inv_r, r1;           // Int 1/R, Int R
    V3 v_inv_r, v_r1;           // Int (rho' - rho)/R, Int (rho' - rho) R
    V3 g_inv_r, g_r1;           // Int grad_r (1/R), Int grad_r R
    V3 rho;                     // projection of r on the plane
};

// ln((R+ + s+)/(R- + s-)), evaluated through the equal form with the larger
// arguments: (R+ + s+)(R+ - s+) = (R- + s-)(R- - s-) = R0^2.
inline double edge_log(double rp, double sp, double rm, double sm) {
    double n1 = rp + sp, d1 = rm + sm, n2 = rm - sm, d2 = rp - sp;
    double v;
    if (std::min(n1, d1) >= std::min(n2, d2)) v = std::log(n1 / d1);
    else v = std::log(n2 / d2);
    return std::isfinite(v) ? v : 0.0;
}

Closed closed_form(const V3 &r, const V3 *p, const V3 &n, bool in_plane) {
    Closed c{};
    double h = in_plane ? 0.0 : dot(r - p[0], n);
    double ah = std::fabs(h);
    c.rho = r - h * n;
    double sum_te_m1 = 0, sum_te1 = 0, sum_beta = 0;
    V3 sm_e1{0, 0, 0}, sm_e3{0, 0, 0}, sm_em1{0, 0, 0};
    for (int i = 0; i < 3; ++i) {
        const V3 &a = p[i], &b = p[(i + 1) % 3];
        V3 s = b - a;
        s = (1.0 / norm(s)) * s;
        V3 mh = cross(s, n);                 // outward in-plane normal of the edge
        double s_lo = dot(a - c.rho, s), s_hi = dot(b - c.rho, s);
        double t = dot(a - c.rho, mh);
        double r0sq = t * t + h * h;
        double R_lo = norm(r - a), R_hi = norm(r - b);
        double e_m1 = edge_log(R_hi, s_hi, R_lo, s_lo);
        double e_1 = 0.5 * (s_hi * R_hi - s_lo * R_lo + r0sq * e_m1);
        double e_3 = 0.25 * (s_hi * R_hi * R_hi * R_hi - s_lo * R_lo * R_lo * R_lo + 3.0 * r0sq * e_1);
        double beta = 0.0;
        if (r0sq + ah * std::min(R_hi, R_lo) > 0)
            beta = std::atan2(t * s_hi, r0sq + ah * R_hi) - std::atan2(t * s_lo, r0sq + ah * R_lo);
        sum_te_m1 += t * e_m1;
        sum_te1 += t * e_1;
        sum_beta += beta;
        for (int j = 0; j < 3; ++j) {
            sm_e1[j] += mh[j] * e_1;
            sm_e3[j] += mh[j] * e_3;
            sm_em1[j] += mh[j] * e_m1;
        }
    }
    c.inv_r = sum_te_m1 - ah * sum_beta;
    c.r1 = (sum_te1 + h * h * c.inv_r) / 3.0;
    double sg = h > 0 ? 1.0 : (h < 0 ? -1.0 : 0.0);
    for (int j = 0; j < 3; ++j) {
        c.v_inv_r[j] = sm_e1[j];
        c.v_r1[j] = sm_e3[j] / 3.0;
        c.g_inv_r[j] = -sm_em1[j] - n[j] * sg * sum_beta;
        c.g_r1[j] = -sm_e1[j] + n[j] * h * c.inv_r;
    }
    return c;
}

inline cd expmj(cd k, double R) {  // exp(-j k R)
    double mag = std::exp(k.imag() * R);
    double ph = k.real() * R;
    return cd(mag * std::cos(ph), -mag * std::sin(ph));
}

}  // namespace

// Local 3x3 interactions of the half-basis functions (r - v_i)/(2A) of test
// triangle P and source triangle Q for wavenumber k:
//   L[i][j] = <h_i, L h_j>, K[i][j] = <h_i, K h_j> (principal value)
// and, when LN != nullptr, the same fields tested with the rotated halves
// t_i = n_P x h_i (eqs. 8-9):
//   LN[i][j] = <t_i, L h_j>, with L h = -j k int h G - (j / k) grad int (div' h) G
//              (t is not divergence-conforming, so the gradient stays on G)
//   KN[i][j] = <t_i, K h_j>  (0 for Q = P: the field of P lies in its plane)
void pair_local(const Mesh &m, int P, int Q, cd k, bool close, cd L[3][3], cd K[3][3], cd (*LN)[3] = nullptr,
                cd (*KN)[3] = nullptr) {
    const TriRule &q = tri_rule();
    const double AP = m.area[P], AQ = m.area[Q];
    const V3 pv[3] = {m.V[m.T[P][0]], m.V[m.T[P][1]], m.V[m.T[P][2]]};
    const V3 qv[3] = {m.V[m.T[Q][0]], m.V[m.T[Q][1]], m.V[m.T[Q][2]]};
    const bool same = (P == Q);
    const cd jk(0.0, 1.0);
    const double inv4pi = 1.0 / (4.0 * PI);
    cd Lacc[3][3] = {}, Kacc[3][3] = {}, LNacc[3][3] = {}, KNacc[3][3] = {};
    const V3 &np = m.normal[P];
    for (int a = 0; a < 7; ++a) {
        const V3 &ra = m.qp[P][a];
        cd Isc = 0;
        cd Ivec[3] = {0, 0, 0}, g[3] = {0, 0, 0};
        for (int b = 0; b < 7; ++b) {
            const V3 &rb = m.qp[Q][b];
            V3 d = ra - rb;
            double R = norm(d);
            double wb = q.w[b] * AQ;
            cd G, gf;
            if (close) {
                if (R > 0) {
                    cd e = expmj(k, R);
                    cd kr = k * R;
                    G = (e - 1.0 + 0.5 * kr * kr) * (inv4pi / R);
                    gf = (-(1.0 + jk * kr) * e + 1.0 + 0.5 * kr * kr) * (inv4pi / (R * R * R));
                } else {
                    G = -jk * k * inv4pi;  // limit of the remainder at R = 0
                    gf = 0.0;
                }
            } else {
                cd e = expmj(k, R);
                G = e * (inv4pi / R);
                gf = -(1.0 + jk * k * R) * e * (inv4pi / (R * R * R));
            }
            Isc += wb * G;
            for (int j = 0; j < 3; ++j) {
                Ivec[j] += wb * G * rb[j];
                g[j] += wb * gf * d[j];
            }
        }
        if (close) {
            Closed c = closed_form(ra, qv, m.normal[Q], same);
            cd k2h = 0.5 * k * k;
            cd ssc = (c.inv_r - k2h * c.r1) * inv4pi;
            Isc += ssc;
            for (int j = 0; j < 3; ++j) {
                Ivec[j] += (c.v_inv_r[j] - k2h * c.v_r1[j]) * inv4pi + c.rho[j] * ssc;
                g[j] += (c.g_inv_r[j] - k2h * c.g_r1[j]) * inv4pi;
            }
        }
        const double wa = q.w[a] * AP;
        for (int i = 0; i < 3; ++i) {
            V3 ri = ra - pv[i];
            for (int jj = 0; jj < 3; ++jj) {
                V3 rj = ra - qv[jj];
                cd dotv = ri[0] * (Ivec[0] - qv[jj][0] * Isc) + ri[1] * (Ivec[1] - qv[jj][1] * Isc) +
                          ri[2] * (Ivec[2] - qv[jj][2] * Isc);
                Lacc[i][jj] += wa * (dotv - (4.0 / (k * k)) * Isc);
                // (r - p_i) . (g x (r - q_j))
                cd cx = g[1] * rj[2] - g[2] * rj[1];
                cd cy = g[2] * rj[0] - g[0] * rj[2];
                cd cz = g[0] * rj[1] - g[1] * rj[0];
                Kacc[i][jj] += wa * (ri[0] * cx + ri[1] * cy + ri[2] * cz);
                if (LN) {
                    // t_i = n_P x (r - p_i) (times 2 A_P);
                    // A_Q L h_j = (-j k / 2)(Ivec - q_j Isc) - (j / k) g
                    const double tx = np[1] * ri[2] - np[2] * ri[1], ty = np[2] * ri[0] - np[0] * ri[2],
                                 tz = np[0] * ri[1] - np[1] * ri[0];
                    const cd lx = (-0.5 * jk * k) * (Ivec[0] - qv[jj][0] * Isc) - (jk / k) * g[0];
                    const cd ly = (-0.5 * jk * k) * (Ivec[1] - qv[jj][1] * Isc) - (jk / k) * g[1];
                    const cd lz = (-0.5 * jk * k) * (Ivec[2] - qv[jj][2] * Isc) - (jk / k) * g[2];
                    LNacc[i][jj] += wa * (tx * lx + ty * ly + tz * lz);
                    KNacc[i][jj] += wa * (tx * cx + ty * cy + tz * cz);
                }
            }
        }
    }
    const cd lf = -jk * k / (4.0 * AP * AQ);
    const double kf = 1.0 / (4.0 * AP * AQ);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            L[i][j] = lf * Lacc[i][j];
            K[i][j] = same ? cd(0.0) : kf * Kacc[i][j];
            if (LN) {
                LN[i][j] = LNacc[i][j] / (2.0 * AP * AQ);
                KN[i][j] = same ? cd(0.0) : kf * KNacc[i][j];
            }
        }
}

// Gram blocks of triangle P's half-bases (the 7-point rule is exact for these
// quadratics): G[i][j] = int_P h_i . h_j, GN[i][j] = int_P h_i . (n_P x h_j).
static void gram_local(const Mesh &m, int P, double G[3][3], double GN[3][3]) {
    const TriRule &q = tri_rule();
    const double A = m.area[P];
    const V3 pv[3] = {m.V[m.T[P][0]], m.V[m.T[P][1]], m.V[m.T[P][2]]};
    const V3 &n = m.normal[P];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) G[i][j] = GN[i][j] = 0.0;
    for (int a = 0; a < 7; ++a) {
        const double w = q.w[a] * A / (4.0 * A * A);
        V3 h[3], nh[3];
        for (int i = 0; i < 3; ++i) {
            h[i] = m.qp[P][a] - pv[i];
            nh[i] = V3{n[1] * h[i][2] - n[2] * h[i][1], n[2] * h[i][0] - n[0] * h[i][2], n[0] * h[i][1] - n[1] * h[i][0]};
        }
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                G[i][j] += w * dot(h[i], h[j]);
                GN[i][j] += w * dot(h[i], nh[j]);
            }
    }
}

static bool close_pair(const Mesh &m, int P, int Q) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            if (m.T[P][i] == m.T[Q][j]) return true;
    double d = norm(m.centroid[P] - m.centroid[Q]);
    return d < 2.0 * std::max(m.maxedge[P], m.maxedge[Q]);
}

NearMatrix near_structure(const Octree &o) {
    NearMatrix Z;
    Z.val_ptr.assign(o.nb + 1, 0);
    Z.col_ptr.assign(o.nb + 1, 0);
    for (int b = 0; b < o.nb; ++b) {
        int nrow = o.bstart[b + 1] - o.bstart[b];
        int ncol = 0;
        for (int q = o.nbr_ptr[b]; q < o.nbr_ptr[b + 1]; ++q) {
            int j = o.nbr_idx[q];
            ncol += o.bstart[j + 1] - o.bstart[j];
        }
        Z.col_ptr[b + 1] = Z.col_ptr[b] + ncol;
        Z.val_ptr[b + 1] = Z.val_ptr[b] + (int64_t)nrow * ncol;
    }
    Z.cols.resize(Z.col_ptr[o.nb]);
    for (int b = 0; b < o.nb; ++b) {
        int c = Z.col_ptr[b];
        for (int q = o.nbr_ptr[b]; q < o.nbr_ptr[b + 1]; ++q) {
            int j = o.nbr_idx[q];
            for (int p = o.bstart[j]; p < o.bstart[j + 1]; ++p) Z.cols[c++] = p;
        }
    }
    return Z;
}

// PMCHWT: per region r bordering both triangles, with region-signed test and
// source halves (factor f), A += f et L, B += f K, C += f L / et.
// JMCFIE / CNF (block [[A, -B], [D, C]], scaled as PMCHWT; JMCFIE is the N
// parts minus the T parts, the sign that lets their identity terms
// reinforce): the N parts with unsigned rotated test halves (factor fn,
// source region-signed), A += fn KN, B -= fn LN / et, D -= fn et LN,
// C += fn KN; the T parts (JMCFIE only, weight ts = -1) with region-signed
// halves, A += ts f L, B += ts f K / et, D += ts f et K, C += ts f L; on
// every triangle the identity terms, A += G, C += G and (JMCFIE)
// B -= ts GM, D += ts GJ with GJ = (et_o - et_p) GN / 2 and
// GM = -(1/et_o - 1/et_p) GN / 2 between front region o and back region p.
NearMatrix fill_near(const Mesh &m, const Octree &o, int form) {
    const bool gen = form != SFMM_FORM_PMCHWT;
    const bool tang = form != SFMM_FORM_CNF;
    const double ts = -1.0;   // weight of the T parts in JMCFIE
    NearMatrix Z = near_structure(o);
    const int64_t nnz = Z.val_ptr[o.nb];
    Z.A.assign(nnz, 0.0);
    Z.B.assign(nnz, 0.0);
    Z.C.assign(nnz, 0.0);
    if (gen) Z.D.assign(nnz, 0.0);

#pragma omp parallel
    {
        std::vector<int> colmap(m.ne, -1);   // canonical edge -> column of the current box
        std::vector<int> rowmap(m.ne, -1);   // canonical edge -> row of the current box
        std::vector<int> tests, sources;
        std::vector<char> seen(m.nt, 0);
#pragma omp for schedule(dynamic, 1)
        for (int b = 0; b < o.nb; ++b) {
            const int nrow = o.bstart[b + 1] - o.bstart[b];
            const int ncol = Z.col_ptr[b + 1] - Z.col_ptr[b];
            const int64_t base = Z.val_ptr[b];
            for (int r = 0; r < nrow; ++r) rowmap[o.order[o.bstart[b] + r]] = r;
            for (int c = 0; c < ncol; ++c) colmap[o.order[Z.cols[Z.col_ptr[b] + c]]] = c;
            tests.clear();
            sources.clear();
            for (int r = 0; r < nrow; ++r) {
                int e = o.order[o.bstart[b] + r];
                for (int i = 0; i < m.nside[e]; ++i) {
                    const int t = m.etri[e][i];
                    if (!(seen[t] & 1)) { seen[t] |= 1; tests.push_back(t); }
                }
            }
            for (int c = 0; c < ncol; ++c) {
                int e = o.order[Z.cols[Z.col_ptr[b] + c]];
                for (int i = 0; i < m.nside[e]; ++i) {
                    const int t = m.etri[e][i];
                    if (!(seen[t] & 2)) { seen[t] |= 2; sources.push_back(t); }
                }
            }
            for (int t : tests) seen[t] = 0;
            for (int t : sources) seen[t] = 0;
            cd L[3][3], K[3][3], LN[3][3], KN[3][3];
            for (int P : tests) {
                for (int Q : sources) {
                    bool close = close_pair(m, P, Q);
                    for (int rr = 0; rr < 2; ++rr) {
                        int r = m.TR[P][rr];
                        if (m.TR[Q][0] != r && m.TR[Q][1] != r) continue;
                        pair_local(m, P, Q, m.k[r], close, L, K, gen ? LN : nullptr, gen ? KN : nullptr);
                        const cd et = m.eta[r];
                        for (int i = 0; i < 3; ++i) {
                            int em = m.tri_edge[P][i];
                            int row = rowmap[em];
                            if (row < 0) continue;
                            double sm = m.tri_region_sign(P, r) * m.tri_sign[P][i] * m.len[em];
                            double smn = m.tri_sign[P][i] * m.len[em];
                            for (int j = 0; j < 3; ++j) {
                                int en = m.tri_edge[Q][j];
                                int col = colmap[en];
                                if (col < 0) continue;
                                double sn = m.tri_region_sign(Q, r) * m.tri_sign[Q][j] * m.len[en];
                                double f = sm * sn;
                                int64_t idx = base + (int64_t)row * ncol + col;
                                if (!gen) {
                                    Z.A[idx] += f * et * L[i][j];
                                    Z.B[idx] += f * K[i][j];
                                    Z.C[idx] += f * L[i][j] / et;
                                    continue;
                                }
                                const double fn = smn * sn;
                                cd a = fn * KN[i][j], b = -fn * LN[i][j] / et, d = -fn * et * LN[i][j];
                                if (tang) {
                                    a += ts * f * L[i][j];
                                    b += ts * f * K[i][j] / et;
                                    d += ts * f * et * K[i][j];
                                }
                                Z.A[idx] += a;
                                Z.B[idx] += b;
                                Z.C[idx] += a;
                                Z.D[idx] += d;
                            }
                        }
                    }
                    if (gen && Q == P) {
                        double G[3][3], GN[3][3];
                        gram_local(m, P, G, GN);
                        const cd eo = m.eta[m.TR[P][0]], ep = m.eta[m.TR[P][1]];
                        const cd wj = tang ? ts * 0.5 * (eo - ep) : cd(0.0);
                        const cd wm = tang ? -ts * 0.5 * (1.0 / eo - 1.0 / ep) : cd(0.0);
                        for (int i = 0; i < 3; ++i) {
                            int em = m.tri_edge[P][i];
                            int row = rowmap[em];
                            if (row < 0) continue;
                            double sm = m.tri_sign[P][i] * m.len[em];
                            for (int j = 0; j < 3; ++j) {
                                int en = m.tri_edge[P][j];
                                int col = colmap[en];
                                if (col < 0) continue;
                                double f = sm * m.tri_sign[P][j] * m.len[en];
                                int64_t idx = base + (int64_t)row * ncol + col;
                                Z.A[idx] += f * G[i][j];
                                Z.C[idx] += f * G[i][j];
                                Z.B[idx] -= f * wm * GN[i][j];
                                Z.D[idx] += f * wj * GN[i][j];
                            }
                        }
                    }
                }
            }
            for (int r = 0; r < nrow; ++r) rowmap[o.order[o.bstart[b] + r]] = -1;
            for (int c = 0; c < ncol; ++c) colmap[o.order[Z.cols[Z.col_ptr[b] + c]]] = -1;
        }
    }
    return Z;
}

}  // namespace sfmm
