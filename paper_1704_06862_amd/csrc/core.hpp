// Host-side data structures of the sfmm library: mesh and RWG table, octree,
// FP64 near-field matrix, ILU(0) factors and MLFMM tables.  Everything here
// is built once by sfmm_setup and then uploaded to the GPU.
#pragma once

#include <array>
#include <complex>
#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/sfmm.h"

namespace sfmm {

using cd = std::complex<double>;
constexpr double PI = 3.14159265358979323846;
constexpr double C0 = 299792458.0;                       // m/s
constexpr double MU0 = 4e-7 * PI * 1.00000000055;        // H/m (CODATA 2018)
constexpr double ETA0 = MU0 * C0;                        // ohm

struct Error : std::runtime_error {
    sfmm_status code;
    Error(sfmm_status c, const std::string &m) : std::runtime_error(m), code(c) {}
};

using V3 = std::array<double, 3>;
inline V3 operator-(const V3 &a, const V3 &b) { return {a[0] - b[0], a[1] - b[1], a[2] - b[2]}; }
inline V3 operator+(const V3 &a, const V3 &b) { return {a[0] + b[0], a[1] + b[1], a[2] + b[2]}; }
inline V3 operator*(double s, const V3 &a) { return {s * a[0], s * a[1], s * a[2]}; }
inline double dot(const V3 &a, const V3 &b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
inline V3 cross(const V3 &a, const V3 &b) {
    return {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
}
inline double norm(const V3 &a) { return std::sqrt(dot(a, a)); }

// Seven-point degree-5 triangle rule (Radon): barycentric nodes and weights.
struct TriRule {
    double bary[7][3];
    double w[7];
    TriRule();
};
const TriRule &tri_rule();

// ---------------------------------------------------------------------------
// Mesh and RWG edges (one body).
struct Mesh {
    int nv = 0, nt = 0, nr = 0, ne = 0;
    std::vector<V3> V;
    std::vector<std::array<int, 3>> T;
    std::vector<std::array<int, 2>> TR;   // (front region, back region)
    std::vector<cd> eps, mu, k, eta;       // per region; eta relative to eta0
    double freq = 0, k0 = 0;
    // triangles
    std::vector<double> area, maxedge;
    std::vector<V3> normal, centroid;
    std::vector<std::array<V3, 7>> qp;     // quadrature nodes
    // edges, canonical order.  An edge carries one half basis function
    // h_t = l / (2 A_t) (r - v_t) (flux out of t across the edge) on each of
    // its nside triangles: two on an interface, three where three regions
    // meet (a junction edge).  Its coefficient there is +1 on a triangle that
    // runs along the edge from the smaller to the larger vertex id (T+), -1
    // otherwise, so f = h_T+ - h_T- on an interface edge.
    std::vector<std::array<int, 2>> ev;    // (min, max) vertex ids
    std::vector<int> nside;
    std::vector<std::array<int, 3>> etri, efree, ecoef;
    std::vector<double> len;
    // per triangle and local vertex i: opposite edge and coefficient of its
    // half basis there
    std::vector<std::array<int, 3>> tri_edge;
    std::vector<std::array<int, 3>> tri_sign;
    // region sign of triangle t for region r (eqs. 12-13, 16): +1 if its
    // normal points into r, -1 if r lies behind it, 0 if t does not border r
    int tri_region_sign(int t, int r) const { return TR[t][0] == r ? 1 : (TR[t][1] == r ? -1 : 0); }
    // Restricted to region r, basis e is s * sum over its triangles t that
    // border r of c_t h_t, with s = edge_region_sign(e, r) and
    // c_t = s * tri_region_sign(t, r) * ecoef[e][t]; for an interface edge s
    // is the interface's region sign and c_t = ecoef.  0 if e does not touch r.
    int edge_region_sign(int e, int r) const {
        for (int i = 0; i < nside[e]; ++i) {
            const int s = tri_region_sign(etri[e][i], r);
            if (s) return s;
        }
        return 0;
    }
};

Mesh build_mesh(const sfmm_body &b);

// ---------------------------------------------------------------------------
// Octree.  Finest boxes are stored in ILU (colour, Morton) order; the
// internal unknown order is box by box, canonical edge order inside a box.
struct LevelBoxes {               // boxes of one region at one level
    double a = 0;                 // box edge
    std::vector<std::array<int, 3>> key;
    std::vector<int> parent;      // index into level - 1 (levels >= 3)
    std::vector<int> child_slot;  // 0..7: octant of this box in its parent
    // children of each box (CSR into level + 1), for the downward pass
    std::vector<int> child_ptr, child_idx;
    // interaction list (CSR): source box index and offset id (dx+3)*49+(dy+3)*7+(dz+3)
    std::vector<int> il_ptr, il_src, il_off;
};

struct RegionTree {               // MLFMM structure of one region
    int region = 0;
    std::vector<int> levels_L;    // truncation order per level (index = level)
    // finest level: boxes that contain edges of this region
    std::vector<int> fbox;        // finest-box id (global) of every region box
    std::vector<int> edge_ptr;    // CSR over region boxes -> positions in edge lists
    std::vector<int> edge_pos;    // internal positions of the region's edges
    std::vector<int> edge_sign;   // region sign of those edges
    std::vector<LevelBoxes> lev;  // index = level (0, 1 unused)
};

struct Octree {
    int nlev = 0, f = 0;          // levels counting the root, finest level index
    double a_f = 0;
    V3 corner{};
    std::vector<std::array<int, 3>> ekey;    // finest key per canonical edge
    int nb = 0;
    std::vector<std::array<int, 3>> bkey;    // per finest box
    std::vector<int> bcolour;
    std::array<int, 9> colour_ptr{};
    std::vector<int> bstart;                 // [nb + 1] internal positions
    std::vector<int> order;                  // internal position -> canonical edge
    std::vector<int> pos;                    // canonical edge -> internal position
    std::vector<int> nbr_ptr, nbr_idx;       // neighbour boxes (incl. self), ascending
    std::vector<RegionTree> regions;
    int64_t near_pairs = 0, trans_pairs = 0;
};

Octree build_octree(const Mesh &m, double finest_box, int n_levels, double digits, int extra);

// ---------------------------------------------------------------------------
// Near-field matrix in box-ELL layout: the rows of finest box b are its edges
// (n_b rows); its columns are the edges of its neighbour boxes in nbr order
// (nc_b columns).  Each edge pair holds the 2x2 block [[A, -B], [D, C]] of the
// scaled system; for PMCHWT D = B and D is not stored.
struct NearMatrix {
    std::vector<int64_t> val_ptr;   // [nb + 1] offset of box b's first entry
    std::vector<int> col_ptr;       // [nb + 1] offset into cols
    std::vector<int> cols;          // internal positions
    std::vector<cd> A, B, C, D;     // D empty: D = B
    const cd &d(int64_t i) const { return D.empty() ? B[i] : D[i]; }
};

// form: SFMM_FORM_PMCHWT, SFMM_FORM_JMCFIE or SFMM_FORM_CNF
NearMatrix fill_near(const Mesh &m, const Octree &o, int form);
// The box-ELL structure alone (pointers and columns, no values).
NearMatrix near_structure(const Octree &o);

// ILU(0) of the near matrix in box-block form, folded for the solves:
//   forward : z_I = Linv_II v_I - sum_{K<I} (Linv_II L_IK) z_K
//   backward: w_I = Uinv_II z_I - sum_{J>I} (Uinv_II U_IJ) w_J
// Each box row is a dense [2 n_I][2 nc] complex block over its own unknowns
// (first) and the unknowns of the lower (forward) or upper (backward)
// neighbour boxes; unknown 2p is J and 2p+1 is M~ of internal position p.
struct IluFactors {
    std::vector<int> fwd_col_ptr, fwd_cols;   // per box: internal positions (own box first)
    std::vector<int> bwd_col_ptr, bwd_cols;
    std::vector<int64_t> fwd_ptr, bwd_ptr;    // value offsets
    std::vector<cd> fwd, bwd;                 // row-major [2n][2nc]
};

// A pivot of modulus at most pivot_tol times the largest entry of its
// diagonal block counts as zero (SFMM_E_BREAKDOWN).
IluFactors factor_ilu(const Mesh &m, const Octree &o, const NearMatrix &Z, double pivot_tol);
// Block-Jacobi: forward rows hold the inverse of each same-box diagonal block
// of the near matrix, backward rows the identity.
IluFactors factor_block_jacobi(const Mesh &m, const Octree &o, const NearMatrix &Z, double pivot_tol);

// Roots (Leja-ordered harmonic Ritz values) of the near-field GMRES polynomial
// preconditioner of the given degree.
// Inverses of the edges' 2x2 near self blocks, [position][4] row-major.
std::vector<cd> edge_block_inverse(const Octree &o, const NearMatrix &Z);
// Roots (Leja order) of the GMRES residual polynomial of D^-1 Z_near
// (D^-1 = dinv; empty dinv: of Z_near itself).
std::vector<cd> poly_roots(const Mesh &m, const Octree &o, const NearMatrix &Z, int degree,
                           const std::vector<cd> &dinv);

// ---------------------------------------------------------------------------
// MLFMM sampling and tables for one region.
struct Sampling {
    int L = 0, nth = 0, nph = 0, K = 0;
    std::vector<double> x, wx;        // Gauss-Legendre nodes in cos(theta), ascending theta
    std::vector<double> w;            // [K] quadrature weight (theta-major)
    std::vector<V3> khat, th, ph;     // [K]
};
Sampling make_sampling(int L);

struct RegionTables {
    cd k, eta;                        // wavenumber, relative impedance
    bool lossy = false;               // Im k != 0: receive patterns stored separately
    std::vector<Sampling> samp;       // per level (2..f)
    std::vector<cd> tx;               // [n_region_edges][2][K_f] transmit patterns (theta, phi)
    std::vector<cd> rx;               // same for receive when lossy
    // JMCFIE / CNF: patterns of the n x f test functions of every region edge
    // (unsigned halves on the region's triangles, rotated by their normals),
    // receive convention when lossy, transmit convention otherwise
    std::vector<cd> nx;
    std::vector<std::vector<cd>> trans;     // per level: [343][K] C_r * w_k * T_L(k; X)
    std::vector<std::vector<double>> ipA, ipB, ipD;  // per level l (l -> l-1 transition, stored at child level l)
    std::vector<std::vector<cd>> shift_up, shift_dn; // per level l: [8][K_{l-1}]
};

RegionTables build_tables(const Mesh &m, const Octree &o, const RegionTree &rt, int form);

}  // namespace sfmm
