// Polynomial preconditioner built from the near-field matrix.
//
// The paper preconditions its Krylov solver with an incomplete LU of the
// near-field matrix.  For the PMCHWT system ILU(0) of the near field is a poor
// approximation of its inverse (its error operator has spectral radius well
// above 1 and restarted GMRES stalls on the 61,440-unknown sphere), while the
// near field itself is an excellent preconditioner.  This builds a fixed
// polynomial p with p(Z_near) ~ Z_near^-1: the residual polynomial of d steps
// of GMRES on Z_near (Loe & Morgan, "Toward efficient polynomial
// preconditioning for GMRES", NLAA 2022):
//   * d steps of Arnoldi (FP64, classical Gram-Schmidt twice) on Z_near from
//     the deterministic start vector v0[i] = exp(2 pi j frac(i g)),
//     g = (sqrt 5 - 1)/2, i = boundary index of the unknown;
//   * roots theta_k = harmonic Ritz values = eigenvalues of
//     H_d + |h_{d+1,d}|^2 H_d^-H e_d e_d^T;
//   * Leja ordering, applied in product form
//       y = 0, q = v;  for k: y += q / theta_k;  q -= Z_near q / theta_k
//     which gives y = p(Z_near) v with 1 - z p(z) = prod_k (1 - z / theta_k).
// The operator is scaled by the inverses of the edges' 2x2 self blocks
// D_m = [[A_mm, -B_mm], [B_mm, C_mm]]: the polynomial is built for
// D^-1 Z_near and applied as p(D^-1 Z_near) D^-1, which puts the J and M
// unknowns of every interface on one scale (with several interfaces and
// high-contrast or lossy media the unscaled polynomial can stall GMRES).
#include <algorithm>
#include <cmath>

#include "core.hpp"

namespace sfmm {

namespace {

// y = Z_near x in internal interleaved order (FP64, host)
void near_apply(const Octree &o, const NearMatrix &Z, const std::vector<cd> &x, std::vector<cd> &y) {
#pragma omp parallel for schedule(dynamic, 8)
    for (int b = 0; b < o.nb; ++b) {
        const int nrow = o.bstart[b + 1] - o.bstart[b];
        const int ncol = Z.col_ptr[b + 1] - Z.col_ptr[b];
        for (int r = 0; r < nrow; ++r) {
            cd e = 0, h = 0;
            const int64_t base = Z.val_ptr[b] + (int64_t)r * ncol;
            for (int c = 0; c < ncol; ++c) {
                const int p = Z.cols[Z.col_ptr[b] + c];
                const cd xj = x[2 * p], xm = x[2 * p + 1];
                e += Z.A[base + c] * xj - Z.B[base + c] * xm;
                h += Z.d(base + c) * xj + Z.C[base + c] * xm;
            }
            y[2 * (o.bstart[b] + r)] = e;
            y[2 * (o.bstart[b] + r) + 1] = h;
        }
    }
}

// y <- D^-1 y, per internal position p (dinv[4p..4p+3] row-major 2x2)
void block_apply(const std::vector<cd> &dinv, std::vector<cd> &y) {
    const int64_t ne = (int64_t)dinv.size() / 4;
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < ne; ++p) {
        const cd e = y[2 * p], h = y[2 * p + 1];
        y[2 * p] = dinv[4 * p] * e + dinv[4 * p + 1] * h;
        y[2 * p + 1] = dinv[4 * p + 2] * e + dinv[4 * p + 3] * h;
    }
}

cd vdot(const std::vector<cd> &a, const std::vector<cd> &b) {
    cd s = 0;
    for (size_t i = 0; i < a.size(); ++i) s += std::conj(a[i]) * b[i];
    return s;
}

// Eigenvalues of a complex upper Hessenberg matrix (row-major n x n) by the
// shifted QR algorithm with Wilkinson shifts and deflation.
std::vector<cd> hessenberg_eigenvalues(std::vector<cd> H, int n) {
    std::vector<cd> ev;
    int hi = n - 1;
    int iter = 0;
    auto at = [&](int i, int j) -> cd & { return H[(size_t)i * n + j]; };
    while (hi >= 0) {
        if (hi == 0) {
            ev.push_back(at(0, 0));
            break;
        }
        // find the start of the active unreduced block
        int lo = hi;
        while (lo > 0) {
            double s = std::abs(at(lo, lo)) + std::abs(at(lo - 1, lo - 1));
            if (std::abs(at(lo, lo - 1)) <= 1e-15 * (s > 0 ? s : 1.0)) {
                at(lo, lo - 1) = 0;
                break;
            }
            --lo;
        }
        if (lo == hi) {
            ev.push_back(at(hi, hi));
            --hi;
            iter = 0;
            continue;
        }
        if (++iter > 300) throw Error(SFMM_E_BREAKDOWN, "QR iteration for harmonic Ritz values did not converge");
        // Wilkinson shift from the trailing 2x2 block
        cd a = at(hi - 1, hi - 1), b = at(hi - 1, hi), c = at(hi, hi - 1), d = at(hi, hi);
        cd tr = a + d, det = a * d - b * c;
        cd disc = std::sqrt(tr * tr - 4.0 * det);
        cd l1 = 0.5 * (tr + disc), l2 = 0.5 * (tr - disc);
        cd mu = (std::abs(l1 - d) < std::abs(l2 - d)) ? l1 : l2;
        if (iter % 11 == 10) mu = d + std::abs(at(hi, hi - 1));   // exceptional shift
        // QR step on the block [lo, hi] via Givens rotations: H - mu I = Q R, H <- R Q + mu I
        const int m = hi - lo + 1;
        std::vector<double> cs(m);
        std::vector<cd> sn(m);
        for (int k = lo; k <= hi; ++k) at(k, k) -= mu;
        for (int k = lo; k < hi; ++k) {
            cd x = at(k, k), y = at(k + 1, k);
            double nx = std::abs(x), ny = std::abs(y);
            double c_, r;
            cd s_;
            if (ny == 0) { c_ = 1; s_ = 0; }
            else if (nx == 0) { c_ = 0; s_ = std::conj(y) / ny; }
            else { r = std::hypot(nx, ny); c_ = nx / r; s_ = (x / nx) * std::conj(y) / r; }
            cs[k - lo] = c_;
            sn[k - lo] = s_;
            for (int j = k; j <= hi; ++j) {   // rows k, k+1
                cd u = at(k, j), v = at(k + 1, j);
                at(k, j) = c_ * u + s_ * v;
                at(k + 1, j) = -std::conj(s_) * u + c_ * v;
            }
        }
        for (int k = lo; k < hi; ++k) {   // R Q: columns k, k+1 times G_k^H
            double c_ = cs[k - lo];
            cd s_ = sn[k - lo];
            for (int i = lo; i <= std::min(k + 1, hi); ++i) {
                cd u = at(i, k), v = at(i, k + 1);
                at(i, k) = c_ * u + std::conj(s_) * v;
                at(i, k + 1) = -s_ * u + c_ * v;
            }
        }
        for (int k = lo; k <= hi; ++k) at(k, k) += mu;
    }
    return ev;
}

}  // namespace

std::vector<cd> edge_block_inverse(const Octree &o, const NearMatrix &Z) {
    std::vector<cd> dinv((size_t)4 * o.bstart[o.nb]);
    for (int b = 0; b < o.nb; ++b) {
        const int nrow = o.bstart[b + 1] - o.bstart[b];
        const int ncol = Z.col_ptr[b + 1] - Z.col_ptr[b];
        for (int r = 0; r < nrow; ++r) {
            const int p = o.bstart[b] + r;
            int c = -1;
            for (int q = 0; q < ncol; ++q)
                if (Z.cols[Z.col_ptr[b] + q] == p) c = q;
            if (c < 0) throw Error(SFMM_E_BREAKDOWN, "edge missing from its own near-field row");
            const int64_t idx = Z.val_ptr[b] + (int64_t)r * ncol + c;
            const cd A = Z.A[idx], B = Z.B[idx], C = Z.C[idx], D = Z.d(idx);
            // [[A, -B], [D, C]]^-1 = [[C, B], [-D, A]] / (A C + B D)
            const cd det = A * C + B * D;
            if (!(std::abs(det) > 0)) throw Error(SFMM_E_BREAKDOWN, "singular edge self block");
            dinv[4 * (size_t)p] = C / det;
            dinv[4 * (size_t)p + 1] = B / det;
            dinv[4 * (size_t)p + 2] = -D / det;
            dinv[4 * (size_t)p + 3] = A / det;
        }
    }
    return dinv;
}

std::vector<cd> poly_roots(const Mesh &m, const Octree &o, const NearMatrix &Z, int degree,
                           const std::vector<cd> &dinv) {
    const int ne = m.ne;
    const int N = 2 * ne;
    const int d = degree;
    if (d < 1 || d > 64) throw Error(SFMM_E_INVALID_ARG, "polynomial degree must be in [1, 64]");
    const double g = 0.5 * (std::sqrt(5.0) - 1.0);
    std::vector<std::vector<cd>> V(d + 1, std::vector<cd>(N));
    for (int e = 0; e < ne; ++e) {
        for (int half = 0; half < 2; ++half) {
            const double i = (double)(half * ne + e);
            const double t = i * g - std::floor(i * g);
            V[0][2 * o.pos[e] + half] = cd(std::cos(2 * PI * t), std::sin(2 * PI * t));
        }
    }
    double n0 = std::sqrt(std::real(vdot(V[0], V[0])));
    for (cd &v : V[0]) v /= n0;
    std::vector<cd> H((size_t)(d + 1) * d, 0.0);
    std::vector<cd> w(N);
    for (int j = 0; j < d; ++j) {
        near_apply(o, Z, V[j], w);
        if (!dinv.empty()) block_apply(dinv, w);
        for (int pass = 0; pass < 2; ++pass)
            for (int i = 0; i <= j; ++i) {
                cd h = vdot(V[i], w);
                H[(size_t)i * d + j] += h;
                for (int t = 0; t < N; ++t) w[t] -= h * V[i][t];
            }
        double hn = std::sqrt(std::real(vdot(w, w)));
        if (!(hn > 0)) throw Error(SFMM_E_BREAKDOWN, "Arnoldi breakdown while building the polynomial");
        H[(size_t)(j + 1) * d + j] = hn;
        for (int t = 0; t < N; ++t) V[j + 1][t] = w[t] / hn;
    }
    // Hh = H_d + |h_{d+1,d}|^2 f e_d^T with H_d^H f = e_d
    std::vector<cd> Hd((size_t)d * d);
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) Hd[(size_t)i * d + j] = H[(size_t)i * d + j];
    {
        // solve H_d^H f = e_d by Gaussian elimination with partial pivoting
        std::vector<cd> A((size_t)d * d), f(d, 0.0);
        for (int i = 0; i < d; ++i)
            for (int j = 0; j < d; ++j) A[(size_t)i * d + j] = std::conj(Hd[(size_t)j * d + i]);
        f[d - 1] = 1.0;
        for (int k = 0; k < d; ++k) {
            int piv = k;
            for (int i = k + 1; i < d; ++i)
                if (std::abs(A[(size_t)i * d + k]) > std::abs(A[(size_t)piv * d + k])) piv = i;
            if (piv != k) {
                for (int j = 0; j < d; ++j) std::swap(A[(size_t)k * d + j], A[(size_t)piv * d + j]);
                std::swap(f[k], f[piv]);
            }
            cd p = A[(size_t)k * d + k];
            if (std::abs(p) == 0) throw Error(SFMM_E_BREAKDOWN, "singular Hessenberg matrix");
            for (int i = k + 1; i < d; ++i) {
                cd fac = A[(size_t)i * d + k] / p;
                for (int j = k; j < d; ++j) A[(size_t)i * d + j] -= fac * A[(size_t)k * d + j];
                f[i] -= fac * f[k];
            }
        }
        for (int i = d - 1; i >= 0; --i) {
            cd s = f[i];
            for (int j = i + 1; j < d; ++j) s -= A[(size_t)i * d + j] * f[j];
            f[i] = s / A[(size_t)i * d + i];
        }
        double h2 = std::norm(H[(size_t)d * d + d - 1]);
        for (int i = 0; i < d; ++i) Hd[(size_t)i * d + d - 1] += h2 * f[i];
    }
    std::vector<cd> th = hessenberg_eigenvalues(Hd, d);
    // Leja ordering: largest modulus first, then maximise the product of distances
    std::vector<cd> out;
    std::vector<bool> used(th.size(), false);
    for (size_t k = 0; k < th.size(); ++k) {
        int best = -1;
        double bv = -1;
        for (size_t i = 0; i < th.size(); ++i) {
            if (used[i]) continue;
            double v = 0;
            if (out.empty()) v = std::abs(th[i]);
            else {
                v = 0;   // log of the product of distances
                for (const cd &s : out) v += std::log(std::abs(th[i] - s) + 1e-300);
            }
            if (best < 0 || v > bv) { best = (int)i; bv = v; }
        }
        used[best] = true;
        out.push_back(th[best]);
    }
    for (const cd &t : out)
        if (!(std::abs(t) > 0)) throw Error(SFMM_E_BREAKDOWN, "zero harmonic Ritz value");
    return out;
}

}  // namespace sfmm
