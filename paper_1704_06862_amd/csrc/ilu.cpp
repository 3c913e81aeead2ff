// ILU(0) of the near-field matrix (the paper's incomplete-LU preconditioner;
// the variant is not stated there, ILU(0) on the near pattern is the reading
// used here), computed in FP64 on the host.
//
// The near pattern is a union of dense blocks between neighbouring finest
// boxes, so scalar ILU(0) in the (colour, Morton, edge, J-before-M) order is
// block ILU(0) with dense box blocks and an exact LU (no pivoting) of every
// diagonal block:
//   for box rows I in order:
//     for lower neighbours K < I:  L_IK = A_IK U_KK^-1,
//                                  A_IJ -= L_IK U_KJ  for J > K neighbour of I and K
//     A_II = L_II U_II;            U_IJ = L_II^-1 A_IJ for J > I
// Boxes of one colour are never neighbours, so each colour is processed in
// parallel.  The factors are then folded for the device solves (core.hpp).
#include <algorithm>
#include <cmath>

#include "core.hpp"

namespace sfmm {

namespace {

using Mat = std::vector<cd>;  // row-major

// X = W U^-1 for upper-triangular U (n x n, packed in LU with leading dim n); W is r x n.
void right_solve_upper(Mat &W, int r, int n, const Mat &LU) {
    for (int i = 0; i < r; ++i) {
        cd *w = &W[(size_t)i * n];
        for (int j = 0; j < n; ++j) {
            cd s = w[j];
            for (int l = 0; l < j; ++l) s -= w[l] * LU[(size_t)l * n + j];
            w[j] = s / LU[(size_t)j * n + j];
        }
    }
}

// C -= A B, A r x k, B k x c (row-major)
void gemm_sub(Mat &C, const Mat &A, const Mat &B, int r, int k, int c) {
    for (int i = 0; i < r; ++i) {
        cd *ci = &C[(size_t)i * c];
        for (int l = 0; l < k; ++l) {
            cd a = A[(size_t)i * k + l];
            if (a == cd(0)) continue;
            const cd *bl = &B[(size_t)l * c];
            for (int j = 0; j < c; ++j) ci[j] -= a * bl[j];
        }
    }
}

void lu_inplace(Mat &A, int n, double pivot_tol) {
    double scale = 0;
    for (const cd &v : A) scale = std::max(scale, std::abs(v));
    for (int k = 0; k < n; ++k) {
        cd piv = A[(size_t)k * n + k];
        if (!(std::abs(piv) > pivot_tol * scale)) throw Error(SFMM_E_BREAKDOWN, "zero pivot in ILU(0)");
        for (int i = k + 1; i < n; ++i) {
            cd f = A[(size_t)i * n + k] / piv;
            A[(size_t)i * n + k] = f;
            if (f == cd(0)) continue;
            for (int j = k + 1; j < n; ++j) A[(size_t)i * n + j] -= f * A[(size_t)k * n + j];
        }
    }
}

// W = L^-1 W for unit lower L packed in LU (n x n); W is n x c.
void left_solve_unit_lower(Mat &W, int n, int c, const Mat &LU) {
    for (int i = 0; i < n; ++i)
        for (int l = 0; l < i; ++l) {
            cd f = LU[(size_t)i * n + l];
            if (f == cd(0)) continue;
            for (int j = 0; j < c; ++j) W[(size_t)i * c + j] -= f * W[(size_t)l * c + j];
        }
}

// W = U^-1 W for upper U packed in LU; W is n x c.
void left_solve_upper(Mat &W, int n, int c, const Mat &LU) {
    for (int i = n - 1; i >= 0; --i) {
        for (int l = i + 1; l < n; ++l) {
            cd f = LU[(size_t)i * n + l];
            if (f == cd(0)) continue;
            for (int j = 0; j < c; ++j) W[(size_t)i * c + j] -= f * W[(size_t)l * c + j];
        }
        cd d = LU[(size_t)i * n + i];
        for (int j = 0; j < c; ++j) W[(size_t)i * c + j] /= d;
    }
}

}  // namespace

IluFactors factor_ilu(const Mesh &m, const Octree &o, const NearMatrix &Z, double pivot_tol) {
    (void)m;
    const int nb = o.nb;
    auto nu = [&](int b) { return 2 * (o.bstart[b + 1] - o.bstart[b]); };
    // blk[I][q]: block with the q-th neighbour of I, [nu(I)][nu(J)] row-major
    std::vector<std::vector<Mat>> blk(nb);
#pragma omp parallel for schedule(dynamic, 4)
    for (int I = 0; I < nb; ++I) {
        const int nrow = o.bstart[I + 1] - o.bstart[I];
        const int ncol = Z.col_ptr[I + 1] - Z.col_ptr[I];
        const int nq = o.nbr_ptr[I + 1] - o.nbr_ptr[I];
        blk[I].resize(nq);
        int c0 = 0;
        for (int q = 0; q < nq; ++q) {
            int J = o.nbr_idx[o.nbr_ptr[I] + q];
            int nJ = o.bstart[J + 1] - o.bstart[J];
            Mat &W = blk[I][q];
            W.assign((size_t)4 * nrow * nJ, 0.0);
            const int ld = 2 * nJ;
            for (int r = 0; r < nrow; ++r)
                for (int c = 0; c < nJ; ++c) {
                    int64_t idx = Z.val_ptr[I] + (int64_t)r * ncol + c0 + c;
                    W[(size_t)(2 * r) * ld + 2 * c] = Z.A[idx];
                    W[(size_t)(2 * r) * ld + 2 * c + 1] = -Z.B[idx];
                    W[(size_t)(2 * r + 1) * ld + 2 * c] = Z.d(idx);
                    W[(size_t)(2 * r + 1) * ld + 2 * c + 1] = Z.C[idx];
                }
            c0 += nJ;
        }
    }
    auto nbr_slot = [&](int K, int J) -> int {
        const int *b = &o.nbr_idx[o.nbr_ptr[K]], *e = &o.nbr_idx[o.nbr_ptr[K + 1]];
        const int *it = std::lower_bound(b, e, J);
        return (it != e && *it == J) ? (int)(it - b) : -1;
    };
    auto self_slot = [&](int I) { return nbr_slot(I, I); };

    bool breakdown = false;
    for (int col = 0; col < 8; ++col) {
#pragma omp parallel for schedule(dynamic, 1)
        for (int I = o.colour_ptr[col]; I < o.colour_ptr[col + 1]; ++I) {
            try {
                const int nI = nu(I);
                const int nq = o.nbr_ptr[I + 1] - o.nbr_ptr[I];
                const int qI = self_slot(I);
                for (int q = 0; q < qI; ++q) {
                    const int K = o.nbr_idx[o.nbr_ptr[I] + q];
                    const int nK = nu(K);
                    const Mat &LUK = blk[K][self_slot(K)];
                    right_solve_upper(blk[I][q], nI, nK, LUK);          // L_IK
                    for (int q2 = q + 1; q2 < nq; ++q2) {
                        const int J = o.nbr_idx[o.nbr_ptr[I] + q2];
                        const int s = nbr_slot(K, J);
                        if (s < 0) continue;
                        gemm_sub(blk[I][q2], blk[I][q], blk[K][s], nI, nK, nu(J));
                    }
                }
                lu_inplace(blk[I][qI], nI, pivot_tol);
                for (int q = qI + 1; q < nq; ++q) {
                    const int J = o.nbr_idx[o.nbr_ptr[I] + q];
                    left_solve_unit_lower(blk[I][q], nI, nu(J), blk[I][qI]);   // U_IJ
                }
            } catch (const Error &) {
#pragma omp critical
                breakdown = true;
            }
        }
        if (breakdown) throw Error(SFMM_E_BREAKDOWN, "zero pivot in ILU(0) of the near-field matrix");
    }

    // fold for the device: forward [Linv | -Linv L_IK ...], backward [Uinv | -Uinv U_IJ ...]
    IluFactors F;
    F.fwd_col_ptr.assign(nb + 1, 0);
    F.bwd_col_ptr.assign(nb + 1, 0);
    F.fwd_ptr.assign(nb + 1, 0);
    F.bwd_ptr.assign(nb + 1, 0);
    for (int I = 0; I < nb; ++I) {
        const int qI = self_slot(I);
        int cf = nu(I) / 2, cb = nu(I) / 2;
        for (int q = 0; q < o.nbr_ptr[I + 1] - o.nbr_ptr[I]; ++q) {
            int J = o.nbr_idx[o.nbr_ptr[I] + q];
            if (q < qI) cf += nu(J) / 2;
            if (q > qI) cb += nu(J) / 2;
        }
        F.fwd_col_ptr[I + 1] = F.fwd_col_ptr[I] + cf;
        F.bwd_col_ptr[I + 1] = F.bwd_col_ptr[I] + cb;
        F.fwd_ptr[I + 1] = F.fwd_ptr[I] + (int64_t)nu(I) * 2 * cf;
        F.bwd_ptr[I + 1] = F.bwd_ptr[I] + (int64_t)nu(I) * 2 * cb;
    }
    F.fwd_cols.resize(F.fwd_col_ptr[nb]);
    F.bwd_cols.resize(F.bwd_col_ptr[nb]);
    F.fwd.assign(F.fwd_ptr[nb], 0.0);
    F.bwd.assign(F.bwd_ptr[nb], 0.0);
#pragma omp parallel for schedule(dynamic, 4)
    for (int I = 0; I < nb; ++I) {
        const int nI = nu(I);
        const int qI = self_slot(I);
        const int nq = o.nbr_ptr[I + 1] - o.nbr_ptr[I];
        const Mat &LU = blk[I][qI];
        // inverses of the unit-lower and upper factors
        Mat Li((size_t)nI * nI, 0.0), Ui((size_t)nI * nI, 0.0);
        for (int i = 0; i < nI; ++i) Li[(size_t)i * nI + i] = Ui[(size_t)i * nI + i] = 1.0;
        left_solve_unit_lower(Li, nI, nI, LU);
        left_solve_upper(Ui, nI, nI, LU);
        const int ldf = 2 * (F.fwd_col_ptr[I + 1] - F.fwd_col_ptr[I]);
        const int ldb = 2 * (F.bwd_col_ptr[I + 1] - F.bwd_col_ptr[I]);
        cd *fw = &F.fwd[F.fwd_ptr[I]];
        cd *bw = &F.bwd[F.bwd_ptr[I]];
        int *fc = &F.fwd_cols[F.fwd_col_ptr[I]];
        int *bc = &F.bwd_cols[F.bwd_col_ptr[I]];
        for (int p = 0; p < nI / 2; ++p) fc[p] = bc[p] = o.bstart[I] + p;
        for (int i = 0; i < nI; ++i)
            for (int j = 0; j < nI; ++j) {
                fw[(size_t)i * ldf + j] = Li[(size_t)i * nI + j];
                bw[(size_t)i * ldb + j] = Ui[(size_t)i * nI + j];
            }
        int cf = nI, cb = nI;
        for (int q = 0; q < nq; ++q) {
            if (q == qI) continue;
            const int J = o.nbr_idx[o.nbr_ptr[I] + q];
            const int nJ = nu(J);
            const Mat &Bq = blk[I][q];
            const Mat &Inv = (q < qI) ? Li : Ui;
            cd *dst = (q < qI) ? fw : bw;
            const int ld = (q < qI) ? ldf : ldb;
            int &c0 = (q < qI) ? cf : cb;
            int *cols = (q < qI) ? fc : bc;
            for (int p = 0; p < nJ / 2; ++p) cols[c0 / 2 + p] = o.bstart[J] + p;
            for (int i = 0; i < nI; ++i)
                for (int j = 0; j < nJ; ++j) {
                    cd s = 0;
                    for (int l = 0; l < nI; ++l) s += Inv[(size_t)i * nI + l] * Bq[(size_t)l * nJ + j];
                    dst[(size_t)i * ld + c0 + j] = -s;
                }
            c0 += nJ;
        }
    }
    return F;
}

}  // namespace sfmm

namespace sfmm {

IluFactors factor_block_jacobi(const Mesh &m, const Octree &o, const NearMatrix &Z, double pivot_tol) {
    (void)m;
    const int nb = o.nb;
    IluFactors F;
    F.fwd_col_ptr.assign(nb + 1, 0);
    F.bwd_col_ptr.assign(nb + 1, 0);
    F.fwd_ptr.assign(nb + 1, 0);
    F.bwd_ptr.assign(nb + 1, 0);
    for (int I = 0; I < nb; ++I) {
        int n = o.bstart[I + 1] - o.bstart[I];
        F.fwd_col_ptr[I + 1] = F.fwd_col_ptr[I] + n;
        F.fwd_ptr[I + 1] = F.fwd_ptr[I] + (int64_t)4 * n * n;
    }
    F.fwd_cols.resize(F.fwd_col_ptr[nb]);
    F.fwd.assign(F.fwd_ptr[nb], 0.0);
    // an exception must not leave an OpenMP region: flag the breakdown and
    // throw after the loop
    bool breakdown = false;
#pragma omp parallel for schedule(dynamic, 4)
    for (int I = 0; I < nb; ++I) {
        const int n = o.bstart[I + 1] - o.bstart[I];
        const int nu = 2 * n;
        const int ncol = Z.col_ptr[I + 1] - Z.col_ptr[I];
        // column offset of the box itself inside its near row
        int c0 = 0;
        for (int q = o.nbr_ptr[I]; q < o.nbr_ptr[I + 1] && o.nbr_idx[q] != I; ++q) {
            int J = o.nbr_idx[q];
            c0 += o.bstart[J + 1] - o.bstart[J];
        }
        std::vector<cd> A((size_t)nu * nu), Inv((size_t)nu * nu, 0.0);
        for (int r = 0; r < n; ++r)
            for (int c = 0; c < n; ++c) {
                int64_t idx = Z.val_ptr[I] + (int64_t)r * ncol + c0 + c;
                A[(size_t)(2 * r) * nu + 2 * c] = Z.A[idx];
                A[(size_t)(2 * r) * nu + 2 * c + 1] = -Z.B[idx];
                A[(size_t)(2 * r + 1) * nu + 2 * c] = Z.d(idx);
                A[(size_t)(2 * r + 1) * nu + 2 * c + 1] = Z.C[idx];
            }
        for (int i = 0; i < nu; ++i) Inv[(size_t)i * nu + i] = 1.0;
        try {
            lu_inplace(A, nu, pivot_tol);
        } catch (const Error &) {
#pragma omp critical
            breakdown = true;
            continue;
        }
        left_solve_unit_lower(Inv, nu, nu, A);
        left_solve_upper(Inv, nu, nu, A);
        for (int p = 0; p < n; ++p) F.fwd_cols[F.fwd_col_ptr[I] + p] = o.bstart[I] + p;
        std::copy(Inv.begin(), Inv.end(), F.fwd.begin() + F.fwd_ptr[I]);
    }
    if (breakdown) throw Error(SFMM_E_BREAKDOWN, "zero pivot in a block-Jacobi diagonal block");
    return F;
}

}  // namespace sfmm
