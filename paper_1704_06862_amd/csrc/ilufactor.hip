// ILU(0) factorisation of the near-field matrix on the device, FP64: the
// same block factorisation as factor_ilu (ilu.cpp) and the same folded form
// for the solves.
//
// The near pattern is a union of dense blocks between neighbouring finest
// boxes, so ILU(0) in the (colour, Morton, edge, J-before-M) order is block
// ILU(0) with dense box blocks and an exact LU (no pivoting) of every
// diagonal block.  Boxes of one colour are never neighbours, so one launch
// per colour factors all of its box rows, one workgroup per box row I:
//   for lower neighbours K < I (ascending):
//       L_IK = A_IK U_KK^-1                      (threads over rows)
//       A_IJ -= L_IK U_KJ  for later neighbours J of I that neighbour K
//   A_II = L_II U_II                             (threads over rows, one
//                                                 barrier per pivot)
//   U_IJ = L_II^-1 A_IJ  for J > I               (threads over columns)
// A pivot of modulus at most pivot_tol times the largest entry of its block
// (taken before the elimination) raises a flag: SFMM_E_BREAKDOWN.
// A final launch folds every box row for the solves:
//   forward  [L_II^-1 | -L_II^-1 L_IK ...],  backward [U_II^-1 | -U_II^-1 U_IJ ...].
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "core.hpp"
#include "device.hpp"
#include "fp64dev.hpp"

namespace sfmm {

namespace {

using namespace fp64;

#define ILCHK(x)                                                                                         \
    do {                                                                                                 \
        hipError_t e_ = (x);                                                                             \
        if (e_ != hipSuccess) throw Error(SFMM_E_DEVICE, std::string("ILU(0) factorisation: ") + hipGetErrorString(e_)); \
    } while (0)

constexpr int FT = 256;   // threads per workgroup

// C (M x N, leading dim ldc) = (overwrite ? 0 : C) + sign * A B, A M x K,
// B K x N; 32 x 32 output tiles through LDS in steps of 16 along K, each
// thread two rows by two columns of a tile.  Every thread of the
// workgroup calls it (it holds barriers).
__device__ void cgemm(zc *C, int ldc, const zc *A, int lda, const zc *B, int ldb, int M, int N, int K, double sign,
                      bool overwrite, zc *sA, zc *sB) {
    const int tid = threadIdx.x;
    const int tr = tid >> 4, tc = tid & 15;
    for (int i0 = 0; i0 < M; i0 += 32)
        for (int j0 = 0; j0 < N; j0 += 32) {
            zc acc[2][2] = {{{0, 0}, {0, 0}}, {{0, 0}, {0, 0}}};
            for (int l0 = 0; l0 < K; l0 += 16) {
                for (int e = tid; e < 512; e += FT) {
                    const int r = e >> 4, c = e & 15;
                    sA[e] = (i0 + r < M && l0 + c < K) ? A[(int64_t)(i0 + r) * lda + l0 + c] : zc{0, 0};
                    const int rb = e >> 5, cb = e & 31;
                    sB[e] = (l0 + rb < K && j0 + cb < N) ? B[(int64_t)(l0 + rb) * ldb + j0 + cb] : zc{0, 0};
                }
                __syncthreads();
#pragma unroll 4
                for (int l = 0; l < 16; ++l) {
                    const zc a0 = sA[(2 * tr) * 16 + l], a1 = sA[(2 * tr + 1) * 16 + l];
                    const zc b0 = sB[l * 32 + 2 * tc], b1 = sB[l * 32 + 2 * tc + 1];
                    acc[0][0] = acc[0][0] + a0 * b0;
                    acc[0][1] = acc[0][1] + a0 * b1;
                    acc[1][0] = acc[1][0] + a1 * b0;
                    acc[1][1] = acc[1][1] + a1 * b1;
                }
                __syncthreads();
            }
            for (int u = 0; u < 2; ++u)
                for (int v = 0; v < 2; ++v) {
                    const int i = i0 + 2 * tr + u, j = j0 + 2 * tc + v;
                    if (i >= M || j >= N) continue;
                    zc &c = C[(int64_t)i * ldc + j];
                    const zc add = sign * acc[u][v];
                    c = overwrite ? add : c + add;
                }
        }
}

struct Blocks {
    const int *bstart, *nbr_ptr, *nbr_idx, *self;   // self: neighbour slot of the box itself
    const int64_t *boff;                            // [nbr_ptr[nb]] element offset of block (I, q)
    zc *w;                                          // all blocks, row-major [nu(I)][nu(J)]
};

__device__ inline int nu(const Blocks &B, int b) { return 2 * (B.bstart[b + 1] - B.bstart[b]); }

// slot of box J among the neighbours of K, -1 if none (ascending lists)
__device__ inline int slot_of(const Blocks &B, int K, int J) {
    int lo = B.nbr_ptr[K], hi = B.nbr_ptr[K + 1] - 1;
    while (lo <= hi) {
        const int mid = (lo + hi) >> 1;
        const int v = B.nbr_idx[mid];
        if (v == J) return mid - B.nbr_ptr[K];
        if (v < J) lo = mid + 1;
        else hi = mid - 1;
    }
    return -1;
}

// Blocks from the near planes: entry (row r, column c) of box I's near rows
// is edge pair (r, c); column c lies in neighbour q's block at column c - c0.
__global__ void __launch_bounds__(FT) k_ilu_blocks(const Blocks B, int nb, const int64_t *__restrict__ val_ptr,
                                                   const int *__restrict__ col_ptr, const zc *__restrict__ A,
                                                   const zc *__restrict__ Bm, const zc *__restrict__ C,
                                                   const zc *__restrict__ D) {
    const int I = blockIdx.x;
    if (I >= nb) return;
    const int nrow = B.bstart[I + 1] - B.bstart[I];
    const int ncol = col_ptr[I + 1] - col_ptr[I];
    const int64_t base = val_ptr[I];
    for (int e = threadIdx.x; e < nrow * ncol; e += FT) {
        const int r = e / ncol, c = e % ncol;
        int q = 0, c0 = 0;
        for (int qq = B.nbr_ptr[I]; qq < B.nbr_ptr[I + 1]; ++qq) {
            const int J = B.nbr_idx[qq];
            const int nJ = B.bstart[J + 1] - B.bstart[J];
            if (c < c0 + nJ) {
                q = qq - B.nbr_ptr[I];
                break;
            }
            c0 += nJ;
        }
        const int J = B.nbr_idx[B.nbr_ptr[I] + q];
        const int ld = nu(B, J);
        const int cc = c - c0;
        zc *w = B.w + B.boff[B.nbr_ptr[I] + q];
        const int64_t idx = base + (int64_t)r * ncol + c;
        const zc b = Bm[idx];
        w[(int64_t)(2 * r) * ld + 2 * cc] = A[idx];
        w[(int64_t)(2 * r) * ld + 2 * cc + 1] = zc{-b.r, -b.i};
        w[(int64_t)(2 * r + 1) * ld + 2 * cc] = D ? D[idx] : b;
        w[(int64_t)(2 * r + 1) * ld + 2 * cc + 1] = C[idx];
    }
}

// One colour: the box rows first_box .. first_box + gridDim.x - 1.
__global__ void __launch_bounds__(FT) k_ilu_rows(const Blocks B, int first_box, double pivot_tol,
                                                 int *__restrict__ breakdown) {
    __shared__ double red[FT];
    __shared__ zc sA[512], sB[512];
    const int I = first_box + blockIdx.x;
    const int tid = threadIdx.x;
    const int nI = nu(B, I);
    const int q0 = B.nbr_ptr[I], nq = B.nbr_ptr[I + 1] - q0, qI = B.self[I];
    for (int q = 0; q < qI; ++q) {
        const int K = B.nbr_idx[q0 + q];
        const int nK = nu(B, K);
        zc *W = B.w + B.boff[q0 + q];
        const zc *U = B.w + B.boff[B.nbr_ptr[K] + B.self[K]];
        for (int i = tid; i < nI; i += FT) {
            zc *wr = W + (int64_t)i * nK;
            for (int j = 0; j < nK; ++j) {
                zc s = wr[j];
                for (int l = 0; l < j; ++l) s = s - wr[l] * U[(int64_t)l * nK + j];
                wr[j] = zdiv(s, U[(int64_t)j * nK + j]);
            }
        }
        __syncthreads();
        for (int q2 = q + 1; q2 < nq; ++q2) {
            const int J = B.nbr_idx[q0 + q2];
            const int s = slot_of(B, K, J);
            if (s < 0) continue;   // the same for every thread
            const int nJ = nu(B, J);
            zc *Cb = B.w + B.boff[q0 + q2];
            const zc *Bb = B.w + B.boff[B.nbr_ptr[K] + s];
            cgemm(Cb, nJ, W, nK, Bb, nJ, nI, nJ, nK, -1.0, false, sA, sB);
        }
        __syncthreads();
    }
    // LU of the diagonal block, rows i > k owned by threads
    zc *Ad = B.w + B.boff[q0 + qI];
    double m = 0;
    for (int e = tid; e < nI * nI; e += FT) m = fmax(m, sqrt(Ad[e].r * Ad[e].r + Ad[e].i * Ad[e].i));
    red[tid] = m;
    __syncthreads();
    for (int h = FT / 2; h > 0; h >>= 1) {
        if (tid < h) red[tid] = fmax(red[tid], red[tid + h]);
        __syncthreads();
    }
    const double scale = red[0];
    for (int k = 0; k < nI; ++k) {
        const zc piv = Ad[(int64_t)k * nI + k];
        if (tid == 0 && !(sqrt(piv.r * piv.r + piv.i * piv.i) > pivot_tol * scale)) atomicOr(breakdown, 1);
        for (int i = k + 1 + tid; i < nI; i += FT) {
            zc *ar = Ad + (int64_t)i * nI;
            const zc f = zdiv(ar[k], piv);
            ar[k] = f;
            for (int j = k + 1; j < nI; ++j) ar[j] = ar[j] - f * Ad[(int64_t)k * nI + j];
        }
        __syncthreads();
    }
    // U_IJ = L_II^-1 A_IJ for the upper neighbours, threads over columns
    for (int q = qI + 1; q < nq; ++q) {
        const int J = B.nbr_idx[q0 + q];
        const int nJ = nu(B, J);
        zc *Cb = B.w + B.boff[q0 + q];
        for (int j = tid; j < nJ; j += FT)
            for (int i = 1; i < nI; ++i) {
                zc s = Cb[(int64_t)i * nJ + j];
                for (int l = 0; l < i; ++l) s = s - Ad[(int64_t)i * nI + l] * Cb[(int64_t)l * nJ + j];
                Cb[(int64_t)i * nJ + j] = s;
            }
    }
}

struct Fold {
    const int64_t *fwd_ptr, *bwd_ptr;
    const int *fwd_col_ptr, *bwd_col_ptr;
    zc *fwd, *bwd;
};

// Folded rows of box I: inverses of the unit-lower and upper factors of the
// diagonal block in the first nI columns, then -L^-1 L_IK and -U^-1 U_IJ.
__global__ void __launch_bounds__(FT) k_ilu_fold(const Blocks B, const Fold F, int nb) {
    __shared__ zc sA[512], sB[512];
    const int I = blockIdx.x;
    if (I >= nb) return;
    const int tid = threadIdx.x;
    const int nI = nu(B, I);
    const int q0 = B.nbr_ptr[I], nq = B.nbr_ptr[I + 1] - q0, qI = B.self[I];
    const zc *LU = B.w + B.boff[q0 + qI];
    const int ldf = 2 * (F.fwd_col_ptr[I + 1] - F.fwd_col_ptr[I]);
    const int ldb = 2 * (F.bwd_col_ptr[I + 1] - F.bwd_col_ptr[I]);
    zc *fw = F.fwd + F.fwd_ptr[I];
    zc *bw = F.bwd + F.bwd_ptr[I];
    for (int j = tid; j < nI; j += FT) {
        // column j of L^-1: x_i = delta_ij - sum_{l<i} L_il x_l
        for (int i = 0; i < nI; ++i) {
            zc s{i == j ? 1.0 : 0.0, 0.0};
            for (int l = j; l < i; ++l) s = s - LU[(int64_t)i * nI + l] * fw[(int64_t)l * ldf + j];
            fw[(int64_t)i * ldf + j] = i < j ? zc{0, 0} : s;
        }
        // column j of U^-1: x_i = (delta_ij - sum_{l>i} U_il x_l) / U_ii
        for (int i = nI - 1; i >= 0; --i) {
            zc s{i == j ? 1.0 : 0.0, 0.0};
            for (int l = i + 1; l <= j; ++l) s = s - LU[(int64_t)i * nI + l] * bw[(int64_t)l * ldb + j];
            bw[(int64_t)i * ldb + j] = i > j ? zc{0, 0} : zdiv(s, LU[(int64_t)i * nI + i]);
        }
    }
    __syncthreads();
    int cf = nI, cb = nI;
    for (int q = 0; q < nq; ++q) {
        if (q == qI) continue;
        const int J = B.nbr_idx[q0 + q];
        const int nJ = nu(B, J);
        const zc *Bq = B.w + B.boff[q0 + q];
        const bool lower = q < qI;
        zc *dst = lower ? fw : bw;
        const int ld = lower ? ldf : ldb;
        const int c0 = lower ? cf : cb;
        cgemm(dst + c0, ld, dst, ld, Bq, nJ, nI, nJ, nI, -1.0, true, sA, sB);
        if (lower) cf += nJ;
        else cb += nJ;
    }
}

template <typename U>
U *dup(const std::vector<U> &v, std::vector<void *> &owned) {
    U *p = nullptr;
    ILCHK(hipMalloc(&p, sizeof(U) * std::max<size_t>(v.size(), 1)));
    owned.push_back(p);
    if (!v.empty()) ILCHK(hipMemcpy(p, v.data(), sizeof(U) * v.size(), hipMemcpyHostToDevice));
    return p;
}

}  // namespace

IluFactors factor_ilu_device(const Octree &o, const NearMatrix &Z, double pivot_tol, int device) {
    const int nb = o.nb;
    auto nub = [&](int b) { return 2 * (o.bstart[b + 1] - o.bstart[b]); };
    std::vector<int> self(nb, -1);
    std::vector<int64_t> boff((size_t)o.nbr_ptr[nb] + 1, 0);
    int64_t total = 0;
    for (int I = 0; I < nb; ++I)
        for (int q = o.nbr_ptr[I]; q < o.nbr_ptr[I + 1]; ++q) {
            const int J = o.nbr_idx[q];
            if (J == I) self[I] = q - o.nbr_ptr[I];
            boff[q] = total;
            total += (int64_t)nub(I) * nub(J);
        }
    for (int I = 0; I < nb; ++I)
        if (self[I] < 0) throw Error(SFMM_E_BREAKDOWN, "box missing from its own neighbour list");
    // folded layout (as in factor_ilu)
    IluFactors F;
    F.fwd_col_ptr.assign(nb + 1, 0);
    F.bwd_col_ptr.assign(nb + 1, 0);
    F.fwd_ptr.assign(nb + 1, 0);
    F.bwd_ptr.assign(nb + 1, 0);
    for (int I = 0; I < nb; ++I) {
        int cf = nub(I) / 2, cb = nub(I) / 2;
        for (int q = 0; q < o.nbr_ptr[I + 1] - o.nbr_ptr[I]; ++q) {
            const int J = o.nbr_idx[o.nbr_ptr[I] + q];
            if (q < self[I]) cf += nub(J) / 2;
            if (q > self[I]) cb += nub(J) / 2;
        }
        F.fwd_col_ptr[I + 1] = F.fwd_col_ptr[I] + cf;
        F.bwd_col_ptr[I + 1] = F.bwd_col_ptr[I] + cb;
        F.fwd_ptr[I + 1] = F.fwd_ptr[I] + (int64_t)nub(I) * 2 * cf;
        F.bwd_ptr[I + 1] = F.bwd_ptr[I] + (int64_t)nub(I) * 2 * cb;
    }
    F.fwd_cols.resize(F.fwd_col_ptr[nb]);
    F.bwd_cols.resize(F.bwd_col_ptr[nb]);
    for (int I = 0; I < nb; ++I) {
        int *fc = &F.fwd_cols[F.fwd_col_ptr[I]];
        int *bc = &F.bwd_cols[F.bwd_col_ptr[I]];
        int cf = 0, cb = 0;
        for (int p = 0; p < nub(I) / 2; ++p) fc[cf++] = bc[cb++] = o.bstart[I] + p;
        for (int q = 0; q < o.nbr_ptr[I + 1] - o.nbr_ptr[I]; ++q) {
            if (q == self[I]) continue;
            const int J = o.nbr_idx[o.nbr_ptr[I] + q];
            for (int p = 0; p < nub(J) / 2; ++p) {
                if (q < self[I]) fc[cf++] = o.bstart[J] + p;
                else bc[cb++] = o.bstart[J] + p;
            }
        }
    }
    F.fwd.assign(F.fwd_ptr[nb], 0.0);
    F.bwd.assign(F.bwd_ptr[nb], 0.0);

    ILCHK(hipSetDevice(device));
    std::vector<void *> owned;
    auto release = [&] {
        for (void *p : owned) (void)hipFree(p);
        owned.clear();
    };
    try {
        Blocks B{};
        B.bstart = dup(o.bstart, owned);
        B.nbr_ptr = dup(o.nbr_ptr, owned);
        B.nbr_idx = dup(o.nbr_idx, owned);
        B.self = dup(self, owned);
        B.boff = dup(boff, owned);
        zc *w = nullptr;
        ILCHK(hipMalloc(&w, sizeof(zc) * std::max<int64_t>(total, 1)));
        owned.push_back(w);
        B.w = w;
        {
            const int64_t nnz = Z.val_ptr[nb];
            auto up = [&](const std::vector<cd> &v) {
                return reinterpret_cast<const zc *>(dup(v, owned));
            };
            const zc *A = up(Z.A), *Bm = up(Z.B), *C = up(Z.C);
            const zc *D = Z.D.empty() ? nullptr : up(Z.D);
            (void)nnz;
            hipLaunchKernelGGL(k_ilu_blocks, dim3(nb), dim3(FT), 0, 0, B, nb, dup(Z.val_ptr, owned),
                               dup(Z.col_ptr, owned), A, Bm, C, D);
            ILCHK(hipGetLastError());
        }
        int *flag = nullptr;
        ILCHK(hipMalloc(&flag, sizeof(int)));
        owned.push_back(flag);
        ILCHK(hipMemset(flag, 0, sizeof(int)));
        for (int c = 0; c < 8; ++c) {
            const int n = o.colour_ptr[c + 1] - o.colour_ptr[c];
            if (n <= 0) continue;
            hipLaunchKernelGGL(k_ilu_rows, dim3(n), dim3(FT), 0, 0, B, o.colour_ptr[c], pivot_tol, flag);
            ILCHK(hipGetLastError());
        }
        int hflag = 0;
        ILCHK(hipMemcpy(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost));
        if (hflag) throw Error(SFMM_E_BREAKDOWN, "zero pivot in ILU(0) of the near-field matrix");
        Fold Fd{};
        Fd.fwd_ptr = dup(F.fwd_ptr, owned);
        Fd.bwd_ptr = dup(F.bwd_ptr, owned);
        Fd.fwd_col_ptr = dup(F.fwd_col_ptr, owned);
        Fd.bwd_col_ptr = dup(F.bwd_col_ptr, owned);
        ILCHK(hipMalloc(&Fd.fwd, sizeof(zc) * std::max<int64_t>(F.fwd_ptr[nb], 1)));
        owned.push_back(Fd.fwd);
        ILCHK(hipMalloc(&Fd.bwd, sizeof(zc) * std::max<int64_t>(F.bwd_ptr[nb], 1)));
        owned.push_back(Fd.bwd);
        hipLaunchKernelGGL(k_ilu_fold, dim3(nb), dim3(FT), 0, 0, B, Fd, nb);
        ILCHK(hipGetLastError());
        ILCHK(hipDeviceSynchronize());
        ILCHK(hipMemcpy(F.fwd.data(), Fd.fwd, sizeof(zc) * F.fwd_ptr[nb], hipMemcpyDeviceToHost));
        ILCHK(hipMemcpy(F.bwd.data(), Fd.bwd, sizeof(zc) * F.bwd_ptr[nb], hipMemcpyDeviceToHost));
    } catch (...) {
        release();
        throw;
    }
    release();
    return F;
}

}  // namespace sfmm
