// Octree of one body: finest boxes, the ILU (colour, Morton) ordering, near
// neighbours and, per region, the MLFMM level structure with interaction lists.
//
// The paper states only that the MLFMM of its ref. [17] accelerates the
// products; these are the standard octree rules of the multilevel fast
// multipole algorithm (Song, Lu, Chew, IEEE TAP 45(10), 1997):
//  * root cube centred on the vertex bounding box, side a_f 2^(levels-1);
//  * a basis function lives in the finest box holding its edge midpoint,
//    key = floor((midpoint - corner) / a_f) clamped to the grid;
//  * near pairs: finest keys differ by at most 1 in every coordinate;
//  * interaction list of box b at level l >= 2: boxes whose parents are
//    neighbours of b's parent but which are not neighbours of b;
//  * truncation order per level from the excess-bandwidth formula
//    L = kd + 1.8 d0^(2/3) (kd)^(1/3), d = sqrt(3) a (box diagonal).
#include <algorithm>
#include <cmath>
#include <unordered_map>

#include "core.hpp"

namespace sfmm {

namespace {

inline uint64_t pack(int x, int y, int z) {
    return ((uint64_t)(uint32_t)x << 42) | ((uint64_t)(uint32_t)y << 21) | (uint64_t)(uint32_t)z;
}

inline int64_t morton(const std::array<int, 3> &k) {
    int64_t code = 0;
    for (int bit = 0; bit < 21; ++bit) {
        code |= (int64_t)((k[0] >> bit) & 1) << (3 * bit + 2);
        code |= (int64_t)((k[1] >> bit) & 1) << (3 * bit + 1);
        code |= (int64_t)((k[2] >> bit) & 1) << (3 * bit);
    }
    return code;
}

int ebf_order(double kd, double d0, int extra) {
    double L = kd + 1.8 * std::pow(d0, 2.0 / 3.0) * std::cbrt(kd);
    return std::max(3, (int)std::ceil(L)) + extra;
}

}  // namespace

Octree build_octree(const Mesh &m, double finest_box, int n_levels, double digits, int extra) {
    Octree o;
    const double lambda0 = C0 / m.freq;
    o.a_f = finest_box > 0 ? finest_box : 0.25 * lambda0;
    V3 lo = m.V[0], hi = m.V[0];
    for (const V3 &v : m.V)
        for (int j = 0; j < 3; ++j) {
            lo[j] = std::min(lo[j], v[j]);
            hi[j] = std::max(hi[j], v[j]);
        }
    double ext = std::max({hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2]});
    if (n_levels <= 0) {
        n_levels = 1;
        while (o.a_f * std::ldexp(1.0, n_levels - 1) < ext * (1.0 - 1e-12)) ++n_levels;
    }
    if (n_levels > 20) throw Error(SFMM_E_INVALID_ARG, "too many octree levels");
    double side = o.a_f * std::ldexp(1.0, n_levels - 1);
    if (side < ext * (1.0 - 1e-9)) throw Error(SFMM_E_INVALID_ARG, "octree root smaller than the body");
    o.nlev = n_levels;
    o.f = n_levels - 1;
    for (int j = 0; j < 3; ++j) o.corner[j] = 0.5 * (lo[j] + hi[j]) - 0.5 * side;
    const int nmax = 1 << o.f;

    o.ekey.resize(m.ne);
    for (int e = 0; e < m.ne; ++e) {
        const V3 &a = m.V[m.ev[e][0]], &b = m.V[m.ev[e][1]];
        for (int j = 0; j < 3; ++j) {
            double mid = 0.5 * (a[j] + b[j]);
            int k = (int)std::floor((mid - o.corner[j]) / o.a_f);
            o.ekey[e][j] = std::min(std::max(k, 0), nmax - 1);
        }
    }
    // finest boxes in (colour, Morton) order
    std::unordered_map<uint64_t, int> boxmap;
    std::vector<std::array<int, 3>> keys;
    for (int e = 0; e < m.ne; ++e) {
        uint64_t p = pack(o.ekey[e][0], o.ekey[e][1], o.ekey[e][2]);
        if (boxmap.emplace(p, (int)keys.size()).second) keys.push_back(o.ekey[e]);
    }
    auto colour = [](const std::array<int, 3> &k) { return (k[0] & 1) * 4 + (k[1] & 1) * 2 + (k[2] & 1); };
    std::vector<int> perm(keys.size());
    for (size_t i = 0; i < perm.size(); ++i) perm[i] = (int)i;
    std::sort(perm.begin(), perm.end(), [&](int a, int b) {
        int ca = colour(keys[a]), cb = colour(keys[b]);
        if (ca != cb) return ca < cb;
        return morton(keys[a]) < morton(keys[b]);
    });
    o.nb = (int)keys.size();
    o.bkey.resize(o.nb);
    o.bcolour.resize(o.nb);
    boxmap.clear();
    for (int i = 0; i < o.nb; ++i) {
        o.bkey[i] = keys[perm[i]];
        o.bcolour[i] = colour(o.bkey[i]);
        boxmap[pack(o.bkey[i][0], o.bkey[i][1], o.bkey[i][2])] = i;
    }
    o.colour_ptr.fill(0);
    for (int i = 0; i < o.nb; ++i) o.colour_ptr[o.bcolour[i] + 1]++;
    for (int c = 0; c < 8; ++c) o.colour_ptr[c + 1] += o.colour_ptr[c];
    // internal order: box by box, canonical edge order inside a box
    std::vector<int> ebox(m.ne);
    o.bstart.assign(o.nb + 1, 0);
    for (int e = 0; e < m.ne; ++e) {
        ebox[e] = boxmap[pack(o.ekey[e][0], o.ekey[e][1], o.ekey[e][2])];
        o.bstart[ebox[e] + 1]++;
    }
    for (int b = 0; b < o.nb; ++b) o.bstart[b + 1] += o.bstart[b];
    o.order.resize(m.ne);
    o.pos.resize(m.ne);
    {
        std::vector<int> fill(o.bstart.begin(), o.bstart.end() - 1);
        for (int e = 0; e < m.ne; ++e) {  // ascending e keeps canonical order inside a box
            int p = fill[ebox[e]]++;
            o.order[p] = e;
            o.pos[e] = p;
        }
    }
    // neighbours (27-stencil, including the box itself), ascending box index
    o.nbr_ptr.assign(o.nb + 1, 0);
    o.nbr_idx.clear();
    o.near_pairs = 0;
    for (int b = 0; b < o.nb; ++b) {
        std::vector<int> nb;
        for (int dx = -1; dx <= 1; ++dx)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dz = -1; dz <= 1; ++dz) {
                    auto it = boxmap.find(pack(o.bkey[b][0] + dx, o.bkey[b][1] + dy, o.bkey[b][2] + dz));
                    if (it != boxmap.end()) nb.push_back(it->second);
                }
        std::sort(nb.begin(), nb.end());
        int nrow = o.bstart[b + 1] - o.bstart[b];
        for (int j : nb) {
            o.nbr_idx.push_back(j);
            o.near_pairs += (int64_t)nrow * (o.bstart[j + 1] - o.bstart[j]);
        }
        o.nbr_ptr[b + 1] = (int)o.nbr_idx.size();
    }

    // per-region MLFMM structures
    const double d0 = digits > 0 ? digits : 3.0;
    o.trans_pairs = 0;
    for (int r = 0; r < m.nr; ++r) {
        RegionTree rt;
        rt.region = r;
        rt.edge_ptr.push_back(0);
        for (int b = 0; b < o.nb; ++b) {
            int cnt = 0;
            for (int p = o.bstart[b]; p < o.bstart[b + 1]; ++p) {
                int s = m.edge_region_sign(o.order[p], r);
                if (s) {
                    rt.edge_pos.push_back(p);
                    rt.edge_sign.push_back(s);
                    ++cnt;
                }
            }
            if (cnt) {
                rt.fbox.push_back(b);
                rt.edge_ptr.push_back((int)rt.edge_pos.size());
            }
        }
        if (rt.fbox.empty()) continue;
        rt.lev.resize(o.f + 1);
        rt.levels_L.assign(o.f + 1, 0);
        for (int l = 2; l <= o.f; ++l) {
            double a = o.a_f * std::ldexp(1.0, o.f - l);
            rt.levels_L[l] = ebf_order(std::abs(m.k[r]) * std::sqrt(3.0) * a, d0, extra);
            rt.lev[l].a = a;
        }
        if (o.f >= 2) {
            LevelBoxes &fl = rt.lev[o.f];
            for (int b : rt.fbox) fl.key.push_back(o.bkey[b]);
            for (int l = o.f; l >= 3; --l) {
                LevelBoxes &cl = rt.lev[l], &pl = rt.lev[l - 1];
                std::unordered_map<uint64_t, int> pm;
                std::vector<int> order_c(cl.key.size());
                // parents in Morton order of their keys
                std::vector<std::array<int, 3>> pk;
                for (auto &k : cl.key) {
                    std::array<int, 3> p = {k[0] >> 1, k[1] >> 1, k[2] >> 1};
                    if (pm.emplace(pack(p[0], p[1], p[2]), 0).second) pk.push_back(p);
                }
                std::sort(pk.begin(), pk.end(), [](const std::array<int, 3> &a, const std::array<int, 3> &b) {
                    return morton(a) < morton(b);
                });
                pl.key = pk;
                for (size_t i = 0; i < pk.size(); ++i) pm[pack(pk[i][0], pk[i][1], pk[i][2])] = (int)i;
                cl.parent.resize(cl.key.size());
                cl.child_slot.resize(cl.key.size());
                for (size_t i = 0; i < cl.key.size(); ++i) {
                    auto &k = cl.key[i];
                    cl.parent[i] = pm[pack(k[0] >> 1, k[1] >> 1, k[2] >> 1)];
                    cl.child_slot[i] = ((k[0] & 1) << 2) | ((k[1] & 1) << 1) | (k[2] & 1);
                }
                pl.child_ptr.assign(pl.key.size() + 1, 0);
                for (int p : cl.parent) pl.child_ptr[p + 1]++;
                for (size_t i = 0; i < pl.key.size(); ++i) pl.child_ptr[i + 1] += pl.child_ptr[i];
                pl.child_idx.resize(cl.key.size());
                std::vector<int> fill(pl.child_ptr.begin(), pl.child_ptr.end() - 1);
                for (size_t i = 0; i < cl.key.size(); ++i) pl.child_idx[fill[cl.parent[i]]++] = (int)i;
            }
            for (int l = 2; l <= o.f; ++l) {
                LevelBoxes &lv = rt.lev[l];
                std::unordered_map<uint64_t, int> km;
                for (size_t i = 0; i < lv.key.size(); ++i) km[pack(lv.key[i][0], lv.key[i][1], lv.key[i][2])] = (int)i;
                lv.il_ptr.assign(lv.key.size() + 1, 0);
                for (size_t i = 0; i < lv.key.size(); ++i) {
                    const auto &k = lv.key[i];
                    int px = k[0] >> 1, py = k[1] >> 1, pz = k[2] >> 1;
                    for (int x = 2 * (px - 1); x <= 2 * (px + 1) + 1; ++x)
                        for (int y = 2 * (py - 1); y <= 2 * (py + 1) + 1; ++y)
                            for (int z = 2 * (pz - 1); z <= 2 * (pz + 1) + 1; ++z) {
                                int dx = k[0] - x, dy = k[1] - y, dz = k[2] - z;
                                if (std::max({std::abs(dx), std::abs(dy), std::abs(dz)}) <= 1) continue;
                                auto it = km.find(pack(x, y, z));
                                if (it == km.end()) continue;
                                lv.il_src.push_back(it->second);
                                lv.il_off.push_back((dx + 3) * 49 + (dy + 3) * 7 + (dz + 3));
                            }
                    lv.il_ptr[i + 1] = (int)lv.il_src.size();
                }
                o.trans_pairs += (int64_t)lv.il_src.size();
            }
        }
        o.regions.push_back(std::move(rt));
    }
    return o;
}

}  // namespace sfmm
