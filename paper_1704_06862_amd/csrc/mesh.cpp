// Mesh validation and the RWG edge table (eq. 22 and Fig. 4 of the paper).
//
// Basis n on edge (a, b), a < b: f_n = +l/(2A+) (r - v+) on T+ (the triangle
// whose CCW order runs a -> b), f_n = -l/(2A-) (r - v-) on T-.  Its divergence
// is +l/A+ and -l/A-, so every basis function carries zero net charge.
//
// Junction edges (three regions meeting along a line, as between the layers
// of a stacked body) carry one such half function on each of their three
// triangles, with the same +1 / -1 rule.  Each region sees two of the three;
// with the region signs of eq. 16 those two form an ordinary RWG function of
// the region's closed boundary, so one J and one M unknown per junction edge
// describe the tangential H and E along the junction line, which are shared
// by all three regions.
#include <algorithm>
#include <cmath>
#include <map>

#include "core.hpp"

namespace sfmm {

TriRule::TriRule() {
    const double s15 = std::sqrt(15.0);
    const double a1 = (6.0 - s15) / 21.0, b1 = (9.0 + 2.0 * s15) / 21.0;
    const double a2 = (6.0 + s15) / 21.0, b2 = (9.0 - 2.0 * s15) / 21.0;
    const double w0 = 9.0 / 40.0, w1 = (155.0 - s15) / 1200.0, w2 = (155.0 + s15) / 1200.0;
    const double nodes[7][3] = {{1.0 / 3, 1.0 / 3, 1.0 / 3}, {a1, a1, b1}, {a1, b1, a1}, {b1, a1, a1},
                                {a2, a2, b2}, {a2, b2, a2}, {b2, a2, a2}};
    const double ws[7] = {w0, w1, w1, w1, w2, w2, w2};
    for (int i = 0; i < 7; ++i) {
        for (int j = 0; j < 3; ++j) bary[i][j] = nodes[i][j];
        w[i] = ws[i];
    }
}

const TriRule &tri_rule() {
    static const TriRule r;
    return r;
}

Mesh build_mesh(const sfmm_body &b) {
    Mesh m;
    if (b.n_vertices < 4 || b.n_triangles < 4 || !b.vertices || !b.triangles || !b.tri_regions)
        throw Error(SFMM_E_INVALID_ARG, "body needs vertices, triangles and tri_regions");
    if (b.n_regions < 2 || !b.eps_r || !b.mu_r) throw Error(SFMM_E_INVALID_ARG, "body needs >= 2 regions with eps_r, mu_r");
    if (!(b.frequency_hz > 0) || !std::isfinite(b.frequency_hz))
        throw Error(SFMM_E_INVALID_ARG, "frequency must be positive and finite");
    m.nv = b.n_vertices;
    m.nt = b.n_triangles;
    m.nr = b.n_regions;
    m.freq = b.frequency_hz;
    m.k0 = 2 * PI * m.freq / C0;
    m.V.resize(m.nv);
    for (int i = 0; i < m.nv; ++i)
        for (int j = 0; j < 3; ++j) {
            m.V[i][j] = b.vertices[3 * i + j];
            if (!std::isfinite(m.V[i][j])) throw Error(SFMM_E_INVALID_ARG, "non-finite vertex coordinate");
        }
    m.T.resize(m.nt);
    m.TR.resize(m.nt);
    for (int t = 0; t < m.nt; ++t) {
        for (int j = 0; j < 3; ++j) {
            int v = b.triangles[3 * t + j];
            if (v < 0 || v >= m.nv) throw Error(SFMM_E_MESH, "triangle references a missing vertex");
            m.T[t][j] = v;
        }
        if (m.T[t][0] == m.T[t][1] || m.T[t][1] == m.T[t][2] || m.T[t][0] == m.T[t][2])
            throw Error(SFMM_E_MESH, "triangle with repeated vertex");
        for (int j = 0; j < 2; ++j) {
            int r = b.tri_regions[2 * t + j];
            if (r < 0 || r >= m.nr) throw Error(SFMM_E_MESH, "triangle region label out of range");
            m.TR[t][j] = r;
        }
        if (m.TR[t][0] == m.TR[t][1]) throw Error(SFMM_E_MESH, "triangle separates a region from itself");
    }
    m.eps.resize(m.nr);
    m.mu.resize(m.nr);
    m.k.resize(m.nr);
    m.eta.resize(m.nr);
    for (int r = 0; r < m.nr; ++r) {
        m.eps[r] = cd(b.eps_r[2 * r], b.eps_r[2 * r + 1]);
        m.mu[r] = cd(b.mu_r[2 * r], b.mu_r[2 * r + 1]);
        if (!std::isfinite(m.eps[r].real()) || !std::isfinite(m.eps[r].imag()) || !std::isfinite(m.mu[r].real()) ||
            !std::isfinite(m.mu[r].imag()))
            throw Error(SFMM_E_INVALID_ARG, "non-finite eps_r or mu_r");
        if (std::abs(m.eps[r]) == 0 || std::abs(m.mu[r]) == 0) throw Error(SFMM_E_INVALID_ARG, "zero eps_r or mu_r");
        // the plane wave (eq. 30) and the far field (eqs. 27-28) live in the
        // unbounded region, taken as vacuum
        if (r == 0 && (m.eps[0] != cd(1.0) || m.mu[0] != cd(1.0)))
            throw Error(SFMM_E_INVALID_ARG, "region 0 (the unbounded exterior) must be vacuum: eps_r = mu_r = 1");
        // principal square roots: Im k <= 0 for passive media under exp(+j w t)
        m.k[r] = m.k0 * std::sqrt(m.eps[r] * m.mu[r]);
        m.eta[r] = std::sqrt(m.mu[r] / m.eps[r]);
    }

    const TriRule &q = tri_rule();
    m.area.resize(m.nt);
    m.maxedge.resize(m.nt);
    m.normal.resize(m.nt);
    m.centroid.resize(m.nt);
    m.qp.resize(m.nt);
    for (int t = 0; t < m.nt; ++t) {
        const V3 &p0 = m.V[m.T[t][0]], &p1 = m.V[m.T[t][1]], &p2 = m.V[m.T[t][2]];
        V3 c = cross(p1 - p0, p2 - p0);
        double n2 = norm(c);
        if (!(n2 > 0)) throw Error(SFMM_E_MESH, "degenerate triangle");
        m.area[t] = 0.5 * n2;
        m.normal[t] = (1.0 / n2) * c;
        m.centroid[t] = (1.0 / 3.0) * (p0 + p1 + p2);
        m.maxedge[t] = std::max({norm(p1 - p0), norm(p2 - p1), norm(p0 - p2)});
        for (int i = 0; i < 7; ++i)
            m.qp[t][i] = q.bary[i][0] * p0 + q.bary[i][1] * p1 + q.bary[i][2] * p2;
    }

    // directed edges: local vertex i is free for the edge (i+1) -> (i+2)
    struct Side { int tri, free, local, dir; };
    std::map<std::pair<int, int>, std::vector<Side>> edges;
    for (int t = 0; t < m.nt; ++t) {
        for (int i = 0; i < 3; ++i) {
            int x = m.T[t][(i + 1) % 3], y = m.T[t][(i + 2) % 3];
            edges[{std::min(x, y), std::max(x, y)}].push_back({t, m.T[t][i], i, x < y ? 1 : -1});
        }
    }
    m.ne = (int)edges.size();
    m.ev.resize(m.ne);
    m.nside.resize(m.ne);
    m.etri.assign(m.ne, {-1, -1, -1});
    m.efree.assign(m.ne, {-1, -1, -1});
    m.ecoef.assign(m.ne, {0, 0, 0});
    m.len.resize(m.ne);
    m.tri_edge.assign(m.nt, {-1, -1, -1});
    m.tri_sign.assign(m.nt, {0, 0, 0});
    int e = 0;
    for (auto &kv : edges) {  // std::map iterates in (min, max) order = canonical order
        std::vector<Side> &sd = kv.second;
        if (sd.size() < 2) throw Error(SFMM_E_MESH, "open surface: an edge with a single triangle");
        if (sd.size() > 3)
            throw Error(SFMM_E_MESH, "an edge shared by more than three triangles (only junctions of three "
                                     "regions are supported)");
        // T+ sides first, each group by triangle index
        std::sort(sd.begin(), sd.end(), [](const Side &a, const Side &b) {
            return a.dir != b.dir ? a.dir > b.dir : a.tri < b.tri;
        });
        // every region that borders the edge sees exactly two of its
        // triangles, and its closed boundary is consistently oriented there:
        // seen from the region, the two run along the edge in opposite
        // directions (sigma_t dir_t = -sigma_t' dir_t').  Then the half
        // bases with coefficients dir restrict to a standard RWG function on
        // every region's boundary (flux out of one triangle into the other).
        std::vector<int> regs;
        for (const Side &a : sd)
            for (int j = 0; j < 2; ++j)
                if (std::find(regs.begin(), regs.end(), m.TR[a.tri][j]) == regs.end()) regs.push_back(m.TR[a.tri][j]);
        for (int r : regs) {
            int cnt = 0, acc = 0;
            for (const Side &a : sd) {
                const int sg = m.tri_region_sign(a.tri, r);
                if (!sg) continue;
                ++cnt;
                acc += sg * a.dir;
            }
            if (cnt != 2)
                throw Error(SFMM_E_MESH, sd.size() == 2 ? "edge between triangles of different interfaces"
                                                        : "junction edge where a region does not see exactly "
                                                          "two of the three triangles");
            if (acc != 0)
                throw Error(SFMM_E_MESH, sd.size() == 2 ? "inconsistent orientation across an edge (or an open "
                                                          "or non-manifold surface)"
                                                        : "inconsistent orientation at a junction edge");
        }
        m.ev[e] = {kv.first.first, kv.first.second};
        m.nside[e] = (int)sd.size();
        for (size_t i = 0; i < sd.size(); ++i) {
            m.etri[e][i] = sd[i].tri;
            m.efree[e][i] = sd[i].free;
            m.ecoef[e][i] = sd[i].dir;
            if (m.tri_edge[sd[i].tri][sd[i].local] >= 0)
                throw Error(SFMM_E_MESH, "triangle with a repeated edge");
            m.tri_edge[sd[i].tri][sd[i].local] = e;
            m.tri_sign[sd[i].tri][sd[i].local] = sd[i].dir;
        }
        m.len[e] = norm(m.V[kv.first.second] - m.V[kv.first.first]);
        ++e;
    }
    return m;
}

}  // namespace sfmm
