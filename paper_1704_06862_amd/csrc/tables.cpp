// MLFMM tables of one region (diagonal-form multilevel fast multipole
// algorithm; the paper uses the MLFMM of its ref. [17] without giving its
// internals, so this follows Coifman, Rokhlin, Wandzura, IEEE APM 35(3), 1993
// and Song, Lu, Chew, IEEE TAP 45(10), 1997, written for exp(+j w t)).
//
// For r in box b (centre c_b) and r' in a well-separated box b' (centre c_b'),
// X = c_b - c_b':
//   G(r, r') = (-jk / 16 pi^2) Int exp(-jk k.(r - c_b)) T_L(k, X) exp(+jk k.(r' - c_b')) d^2k
//   T_L(k, X) = sum_{l<=L} (-j)^l (2l+1) h_l^(2)(k|X|) P_l(k . X/|X|)
// Substituting into L and K of eqs. 5-6 (the scalar-potential term turns into
// the transverse projection (I - kk) after integrating by parts):
//   L[m,n] = C Int R_m . (I - kk) F_n T_L,   K[m,n] = C Int R_m . (k x F_n) T_L,
//   C = -k^2 / (16 pi^2),
//   F_n(k) = Int f_n(r') exp(+jk k.(r' - c)) dS'   (transmit pattern)
//   R_m(k) = Int f_m(r)  exp(-jk k.(r - c)) dS    (receive pattern; conj(F_m) for real k)
// so one transverse outgoing pattern per box and region,
//   S = s_n [ et (I - kk) F_n J_n - k x F_n M~_n ],
// feeds both rows: E_m = C Int R_m . T S,  H_m = (C / et) Int R_m . k x (T S).
// The sphere is sampled with L+1 Gauss-Legendre nodes in cos(theta) and
// 2(L+1) uniform nodes in phi; the translation tables fold in C and the
// quadrature weight.  Between levels, patterns are interpolated in theta and
// then phi; the theta/phi components of a smooth tangential field are, per
// azimuthal order m, sin(theta) times a polynomial in cos(theta) for even m
// and a polynomial for odd m, so the even and odd parts (paired through
// phi and phi + pi) get their own Lagrange matrices, and phi uses
// trigonometric interpolation.  Anterpolation is the exact transpose.
#include <algorithm>
#include <cmath>
#include <omp.h>

#include "core.hpp"

namespace sfmm {

namespace {

void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w) {
    // Newton iteration on P_n from the usual initial guesses; nodes come out
    // in descending cos(theta), i.e. ascending theta.
    x.resize(n);
    w.resize(n);
    for (int i = 0; i < n; ++i) {
        double z = std::cos(PI * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double pm1 = 1.0, p = z;                 // P_0, P_1
            for (int l = 2; l <= n; ++l) {
                double pn = ((2 * l - 1) * z * p - (l - 1) * pm1) / l;
                pm1 = p;
                p = pn;
            }
            if (n == 1) pm1 = 1.0;
            dp = n * (z * p - pm1) / (z * z - 1.0);  // P_n'(z)
            double dz = p / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-15) break;
        }
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

// spherical Hankel functions of the second kind, orders 0..L, complex argument
void hankel2(int L, cd z, std::vector<cd> &h) {
    h.assign(L + 1, 0.0);
    const cd j(0.0, 1.0);
    cd e = std::exp(-j * z);
    h[0] = j * e / z;
    if (L >= 1) h[1] = e * (j / (z * z) - 1.0 / z);
    for (int l = 1; l < L; ++l) h[l + 1] = (2.0 * l + 1.0) / z * h[l] - h[l - 1];
}

}  // namespace

Sampling make_sampling(int L) {
    Sampling s;
    s.L = L;
    s.nth = L + 1;
    s.nph = 2 * (L + 1);
    s.K = s.nth * s.nph;
    gauss_legendre(s.nth, s.x, s.wx);
    s.w.resize(s.K);
    s.khat.resize(s.K);
    s.th.resize(s.K);
    s.ph.resize(s.K);
    for (int i = 0; i < s.nth; ++i) {
        double ct = s.x[i], st = std::sqrt(std::max(0.0, 1.0 - ct * ct));
        for (int jj = 0; jj < s.nph; ++jj) {
            double phi = 2.0 * PI * jj / s.nph;
            double cp = std::cos(phi), sp = std::sin(phi);
            int k = i * s.nph + jj;
            s.w[k] = s.wx[i] * 2.0 * PI / s.nph;
            s.khat[k] = {st * cp, st * sp, ct};
            s.th[k] = {ct * cp, ct * sp, -st};
            s.ph[k] = {-sp, cp, 0.0};
        }
    }
    return s;
}

RegionTables build_tables(const Mesh &m, const Octree &o, const RegionTree &rt, int form) {
    RegionTables t;
    const int r = rt.region;
    t.k = m.k[r];
    t.eta = m.eta[r];
    t.lossy = t.k.imag() != 0.0;
    const int f = o.f;
    if (f < 2) return t;
    t.samp.resize(f + 1);
    for (int l = 2; l <= f; ++l) t.samp[l] = make_sampling(rt.levels_L[l]);
    const cd j(0.0, 1.0);
    const cd k = t.k;

    // transmit (and, for complex k, receive) patterns of every region edge
    // about its finest-box centre
    const Sampling &sf = t.samp[f];
    const int ned = (int)rt.edge_pos.size();
    const int Kf = sf.K;
    t.tx.assign((size_t)ned * 2 * Kf, 0.0);
    if (t.lossy) t.rx.assign((size_t)ned * 2 * Kf, 0.0);
    const bool ntest = form != SFMM_FORM_PMCHWT;
    if (ntest) t.nx.assign((size_t)ned * 2 * Kf, 0.0);
    const TriRule &q = tri_rule();
    const int nrb = (int)rt.fbox.size();
#pragma omp parallel for schedule(dynamic, 4)
    for (int ib = 0; ib < nrb; ++ib) {
        const int b = rt.fbox[ib];
        V3 c;
        for (int d = 0; d < 3; ++d) c[d] = o.corner[d] + (o.bkey[b][d] + 0.5) * o.a_f;
        for (int ie = rt.edge_ptr[ib]; ie < rt.edge_ptr[ib + 1]; ++ie) {
            const int e = o.order[rt.edge_pos[ie]];
            // 14 weighted vector samples of f_e restricted to the region (its
            // two triangles there; the region sign stays in edge_sign)
            V3 fv[14], pts[14], nv[14];
            double wq[14];
            const int es = rt.edge_sign[ie];
            int side = 0;
            for (int i = 0; i < m.nside[e]; ++i) {
                const int tri = m.etri[e][i];
                const int rs = m.tri_region_sign(tri, rt.region);
                if (!rs) continue;
                if (side == 2) throw Error(SFMM_E_MESH, "edge with more than two triangles in one region");
                const double coef = es * rs * m.ecoef[e][i] * m.len[e] / (2.0 * m.area[tri]);
                for (int a = 0; a < 7; ++a) {
                    pts[side * 7 + a] = m.qp[tri][a] - c;
                    fv[side * 7 + a] = coef * (m.qp[tri][a] - m.V[m.efree[e][i]]);
                    // n x f with the unsigned half (no region or edge sign)
                    const V3 h = (m.ecoef[e][i] * m.len[e] / (2.0 * m.area[tri])) * (m.qp[tri][a] - m.V[m.efree[e][i]]);
                    const V3 &n = m.normal[tri];
                    nv[side * 7 + a] = V3{n[1] * h[2] - n[2] * h[1], n[2] * h[0] - n[0] * h[2], n[0] * h[1] - n[1] * h[0]};
                    wq[side * 7 + a] = q.w[a] * m.area[tri];
                }
                ++side;
            }
            if (side != 2) throw Error(SFMM_E_MESH, "region edge without two triangles in the region");
            cd *tx = &t.tx[(size_t)ie * 2 * Kf];
            cd *rx = t.lossy ? &t.rx[(size_t)ie * 2 * Kf] : nullptr;
            for (int kk = 0; kk < Kf; ++kk) {
                cd Ft = 0, Fp = 0, Rt = 0, Rp = 0;
                for (int s = 0; s < 14; ++s) {
                    cd ph = std::exp(j * k * dot(sf.khat[kk], pts[s]));
                    double ft = dot(sf.th[kk], fv[s]) * wq[s], fp = dot(sf.ph[kk], fv[s]) * wq[s];
                    Ft += ft * ph;
                    Fp += fp * ph;
                    if (rx) {
                        cd phr = std::exp(-j * k * dot(sf.khat[kk], pts[s]));
                        Rt += ft * phr;
                        Rp += fp * phr;
                    }
                }
                tx[kk] = Ft;
                tx[Kf + kk] = Fp;
                if (rx) {
                    rx[kk] = Rt;
                    rx[Kf + kk] = Rp;
                }
            }
            if (ntest) {
                cd *nx = &t.nx[(size_t)ie * 2 * Kf];
                const double sg = t.lossy ? -1.0 : 1.0;   // receive: exp(-j k khat.r)
                for (int kk = 0; kk < Kf; ++kk) {
                    cd Nt = 0, Np = 0;
                    for (int s = 0; s < 14; ++s) {
                        cd ph = std::exp(sg * j * k * dot(sf.khat[kk], pts[s]));
                        Nt += dot(sf.th[kk], nv[s]) * wq[s] * ph;
                        Np += dot(sf.ph[kk], nv[s]) * wq[s] * ph;
                    }
                    nx[kk] = Nt;
                    nx[Kf + kk] = Np;
                }
            }
        }
    }

    // translation tables per level: [343][K]
    const cd C = -k * k / (16.0 * PI * PI);
    t.trans.resize(f + 1);
    for (int l = 2; l <= f; ++l) {
        const Sampling &s = t.samp[l];
        const double a = rt.lev[l].a;
        std::vector<cd> &T = t.trans[l];
        T.assign((size_t)343 * s.K, 0.0);
#pragma omp parallel for schedule(dynamic, 4)
        for (int id = 0; id < 343; ++id) {
            int dx = id / 49 - 3, dy = (id / 7) % 7 - 3, dz = id % 7 - 3;
            if (std::max({std::abs(dx), std::abs(dy), std::abs(dz)}) <= 1) continue;
            V3 X = {dx * a, dy * a, dz * a};
            double Xn = norm(X);
            V3 Xh = (1.0 / Xn) * X;
            std::vector<cd> h;
            hankel2(s.L, k * Xn, h);
            std::vector<cd> coef(s.L + 1);
            cd mj(1.0, 0.0);
            for (int ll = 0; ll <= s.L; ++ll) {
                coef[ll] = mj * (2.0 * ll + 1.0) * h[ll];
                mj *= cd(0.0, -1.0);
            }
            for (int kk = 0; kk < s.K; ++kk) {
                double x = dot(s.khat[kk], Xh);
                double p0 = 1.0, p1 = x;
                cd sum = coef[0];
                if (s.L >= 1) sum += coef[1] * x;
                for (int ll = 1; ll < s.L; ++ll) {
                    double p2 = ((2 * ll + 1) * x * p1 - ll * p0) / (ll + 1);
                    p0 = p1;
                    p1 = p2;
                    sum += coef[ll + 1] * p2;
                }
                T[(size_t)id * s.K + kk] = C * s.w[kk] * sum;
            }
        }
    }

    // interpolation child level l -> parent level l-1, and shift phases
    t.ipA.resize(f + 1);
    t.ipB.resize(f + 1);
    t.ipD.resize(f + 1);
    t.shift_up.resize(f + 1);
    t.shift_dn.resize(f + 1);
    for (int l = 3; l <= f; ++l) {
        const Sampling &c = t.samp[l], &p = t.samp[l - 1];
        std::vector<double> E((size_t)p.nth * c.nth);
        for (int I = 0; I < p.nth; ++I)
            for (int i = 0; i < c.nth; ++i) {
                double v = 1.0;
                for (int jj = 0; jj < c.nth; ++jj)
                    if (jj != i) v *= (p.x[I] - c.x[jj]) / (c.x[i] - c.x[jj]);
                E[(size_t)I * c.nth + i] = v;
            }
        std::vector<double> &A = t.ipA[l], &B = t.ipB[l], &D = t.ipD[l];
        A.resize(E.size());
        B.resize(E.size());
        for (int I = 0; I < p.nth; ++I) {
            double sI = std::sqrt(std::max(0.0, 1.0 - p.x[I] * p.x[I]));
            for (int i = 0; i < c.nth; ++i) {
                double si = std::sqrt(std::max(0.0, 1.0 - c.x[i] * c.x[i]));
                double e = E[(size_t)I * c.nth + i];
                double es = sI * e / si;
                A[(size_t)I * c.nth + i] = 0.5 * (es + e);
                B[(size_t)I * c.nth + i] = 0.5 * (es - e);
            }
        }
        D.resize((size_t)p.nph * c.nph);
        const int N = c.nph;
        for (int J = 0; J < p.nph; ++J)
            for (int jj = 0; jj < N; ++jj) {
                double x = 2.0 * PI * J / p.nph - 2.0 * PI * jj / N;
                double v = 1.0 + std::cos((N / 2) * x);
                for (int mm = 1; mm < N / 2; ++mm) v += 2.0 * std::cos(mm * x);
                D[(size_t)J * N + jj] = v / N;
            }
        // child centre minus parent centre for octant (sx, sy, sz): (2s - 1) a_child / 2
        const double ac = rt.lev[l].a;
        t.shift_up[l].resize((size_t)8 * p.K);
        t.shift_dn[l].resize((size_t)8 * p.K);
        for (int oct = 0; oct < 8; ++oct) {
            V3 d = {((oct >> 2) & 1 ? 0.5 : -0.5) * ac, ((oct >> 1) & 1 ? 0.5 : -0.5) * ac,
                    (oct & 1 ? 0.5 : -0.5) * ac};
            for (int kk = 0; kk < p.K; ++kk) {
                double kd = dot(p.khat[kk], d);
                t.shift_up[l][(size_t)oct * p.K + kk] = std::exp(j * k * kd);
                t.shift_dn[l][(size_t)oct * p.K + kk] = std::exp(-j * k * kd);
            }
        }
    }
    return t;
}

}  // namespace sfmm
