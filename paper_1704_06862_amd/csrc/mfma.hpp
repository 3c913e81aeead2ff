// Matrix-core (MFMA) kernels for batched right-hand sides on gfx950.
//
// With R right-hand sides in the internal RHS-minor layout, the near-field
// product of one finest box is a dense complex GEMM
//     [E rows; H rows] (2 n_b x R) = [[A, -B], [B, C]] (2 n_b x 2 n_c) [J; M] (2 n_c x R)
// so it runs on the matrix cores: rows in blocks of 16 (the M dimension),
// right-hand sides in blocks of 16 (N), columns along K.  Two arithmetic
// variants share the tiling:
//   FP32       v_mfma_f32_16x16x4_f32, K = 4 columns per step;
//   BF16-split every FP32 operand v is carried as hi = bf16(v) and
//              lo = bf16(v - hi); a product is hi*hi + hi*lo + lo*hi on
//              v_mfma_f32_16x16x32_bf16 (K = 32 per step) with FP32
//              accumulation, about 16 significant bits per operand.
// Operand lane layouts (16x16 output block, lane l in 0..63):
//   A (matrix)  row l % 16, K index (l / 16) * E + e   (E = 1 or 8 elements)
//   B (vectors) column l % 16, same K index
//   D           row 4 (l / 16) + v, column l % 16, v = 0..3
// The matrix is stored once in this tile order at setup (zero padding), so
// every matrix load is a contiguous 64-lane access.
#pragma once

#include "kernels.hpp"

namespace sfmm {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int MMA_WAVES = 4;   // waves per tile workgroup; they split the K steps

// bf16 rounding (to nearest even) of v and of the remainder v - hi
__device__ __forceinline__ void split_bf16(float v, __bf16 &hi, __bf16 &lo) {
    hi = (__bf16)v;
    lo = (__bf16)(v - (float)hi);
}

typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

// sign flip of eight bf16 values (exact)
__device__ __forceinline__ bf16x8 neg8(bf16x8 v) {
    u16x8 u = __builtin_bit_cast(u16x8, v);
    u ^= (unsigned short)0x8000;
    return __builtin_bit_cast(bf16x8, u);
}

__device__ __forceinline__ void mma_f32(f32x4 &c, float a, float b) {
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
// hi*hi + hi*lo + lo*hi
__device__ __forceinline__ void mma_split(f32x4 &c, const bf16x8 &ah, const bf16x8 &al, const bf16x8 &bh,
                                          const bf16x8 &bl) {
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, c, 0, 0, 0);
}

// Near-field product on the matrix cores for R <= 16 * NT right-hand sides.
// One workgroup per tile (box b, 16-row block starting at row0), tiles
// renumbered so that each XCD takes a contiguous range; the 4 waves
// take every 4th K step and their partial sums are added through LDS.
// vals: FP32: three planes (A, B, C) of cx<float>[nsteps][64];
//       split: twelve planes (A, B, C) x (re hi, re lo, im hi, im lo) of
//       bf16x8[nsteps][64].
// GEN (JMCFIE / CNF): a fourth plane D (or four more split planes) holds
// the H-row J coefficient of the block [[A, -B], [D, C]]; otherwise D = B.
// POLY as in k_near: with Q = Z_near X, acc += X / theta, Y = X - Q / theta.
template <int NT, bool SPLIT, bool POLY, bool GEN>
__global__ void __launch_bounds__(64 * MMA_WAVES)
    k_near_mma(int R, const int *__restrict__ tile_box, const int *__restrict__ tile_row0,
               const int64_t *__restrict__ tile_step, const int *__restrict__ bstart, const int *__restrict__ col_ptr,
               const int *__restrict__ cols, const void *__restrict__ vals, int64_t nsteps,
               const cx<float> *__restrict__ x, cx<float> *__restrict__ y, cx<float> *__restrict__ acc,
               cx<float> inv_theta, int write_y, const cx<float> *__restrict__ dinv, int ntiles) {
    __shared__ f32x4 red[MMA_WAVES - 1][NT * 4][64];
    // each XCD takes a contiguous range of tiles (neighbouring boxes, whose
    // column lists overlap, then share that XCD's L2); the grid is 8 per
    const int per = (ntiles + 7) / 8;
    const int t = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    if (t >= ntiles) return;
    const int b = tile_box[t], row0 = tile_row0[t];
    const int r0 = bstart[b], nrow = bstart[b + 1] - r0;
    const int c0 = col_ptr[b], ncol = col_ptr[b + 1] - c0;
    const int64_t st0 = tile_step[t];
    const int nst = (int)(tile_step[t + 1] - st0);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int lr = lane & 15, lg = lane >> 4;
    f32x4 aEr[NT], aEi[NT], aHr[NT], aHi[NT];
#pragma unroll
    for (int n = 0; n < NT; ++n) aEr[n] = aEi[n] = aHr[n] = aHi[n] = f32x4{0, 0, 0, 0};

    for (int s = wave; s < nst; s += MMA_WAVES) {
        const int64_t vi = (st0 + s) * 64 + lane;
        if constexpr (!SPLIT) {
            const cx<float> *V = reinterpret_cast<const cx<float> *>(vals);
            const cx<float> a = V[vi], bb = V[nsteps * 64 + vi], c = V[2 * nsteps * 64 + vi];
            const cx<float> d = GEN ? V[3 * nsteps * 64 + vi] : bb;
            const int col = 4 * s + lg;
            const int p = col < ncol ? cols[c0 + col] : -1;
            const float nay = -a.y, nbx = -bb.x, nby = -bb.y, ncy = -c.y, ndy = -d.y;
#pragma unroll
            for (int n = 0; n < NT; ++n) {
                const int rhs = 16 * n + lr;
                cx<float> xj = {0, 0}, xm = {0, 0};
                if (p >= 0 && rhs < R) {
                    xj = x[(int64_t)(2 * p) * R + rhs];
                    xm = x[(int64_t)(2 * p + 1) * R + rhs];
                }
                // E = A xJ - B xM ; H = D xJ + C xM
                mma_f32(aEr[n], a.x, xj.x);
                mma_f32(aEr[n], nay, xj.y);
                mma_f32(aEr[n], nbx, xm.x);
                mma_f32(aEr[n], bb.y, xm.y);
                mma_f32(aEi[n], a.x, xj.y);
                mma_f32(aEi[n], a.y, xj.x);
                mma_f32(aEi[n], nbx, xm.y);
                mma_f32(aEi[n], nby, xm.x);
                mma_f32(aHr[n], d.x, xj.x);
                mma_f32(aHr[n], ndy, xj.y);
                mma_f32(aHr[n], c.x, xm.x);
                mma_f32(aHr[n], ncy, xm.y);
                mma_f32(aHi[n], d.x, xj.y);
                mma_f32(aHi[n], d.y, xj.x);
                mma_f32(aHi[n], c.x, xm.y);
                mma_f32(aHi[n], c.y, xm.x);
            }
        } else {
            // POLY (the polynomial preconditioner): vals holds only the
            // bfloat16 values, compact planes (A, B, C[, D]) x (re, im), and
            // each step takes two matrix-core products instead of three
            constexpr bool AHI = POLY;
            const bf16x8 *V = reinterpret_cast<const bf16x8 *>(vals);
            const int64_t pl = nsteps * 64;
            const bf16x8 z8 = {};
            constexpr int H = AHI ? 1 : 2;   // plane stride of the hi parts
            const bf16x8 arh = V[vi], aih = V[H * pl + vi], brh = V[2 * H * pl + vi], bih = V[3 * H * pl + vi];
            const bf16x8 crh = V[4 * H * pl + vi], cih = V[5 * H * pl + vi];
            const bf16x8 arl = AHI ? z8 : V[pl + vi], ail = AHI ? z8 : V[3 * pl + vi];
            const bf16x8 brl = AHI ? z8 : V[5 * pl + vi], bil = AHI ? z8 : V[7 * pl + vi];
            const bf16x8 crl = AHI ? z8 : V[9 * pl + vi], cil = AHI ? z8 : V[11 * pl + vi];
            const bf16x8 drh = GEN ? V[6 * H * pl + vi] : brh, drl = GEN ? (AHI ? z8 : V[13 * pl + vi]) : brl;
            const bf16x8 dih = GEN ? V[7 * H * pl + vi] : bih, dil = GEN ? (AHI ? z8 : V[15 * pl + vi]) : bil;
            auto mma_split = [](f32x4 &c, const bf16x8 &ah, const bf16x8 &al, const bf16x8 &bh, const bf16x8 &bl) {
                if constexpr (AHI) {
                    (void)al;
                    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, c, 0, 0, 0);
                    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, c, 0, 0, 0);
                } else {
                    sfmm::mma_split(c, ah, al, bh, bl);
                }
            };
            const bf16x8 naih = neg8(aih), nail = neg8(ail), nbrh = neg8(brh), nbrl = neg8(brl);
            const bf16x8 nbih = neg8(bih), nbil = neg8(bil), ncih = neg8(cih), ncil = neg8(cil);
            const bf16x8 ndih = neg8(dih), ndil = neg8(dil);
            const int colb = 32 * s + 8 * lg;
            int p[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) p[e] = colb + e < ncol ? cols[c0 + colb + e] : -1;
#pragma unroll
            for (int n = 0; n < NT; ++n) {
                const int rhs = 16 * n + lr;
                bf16x8 jrh, jrl, jih, jil, mrh, mrl, mih, mil;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    cx<float> xj = {0, 0}, xm = {0, 0};
                    if (p[e] >= 0 && rhs < R) {
                        xj = x[(int64_t)(2 * p[e]) * R + rhs];
                        xm = x[(int64_t)(2 * p[e] + 1) * R + rhs];
                    }
                    __bf16 h, l;
                    split_bf16(xj.x, h, l);
                    jrh[e] = h;
                    jrl[e] = l;
                    split_bf16(xj.y, h, l);
                    jih[e] = h;
                    jil[e] = l;
                    split_bf16(xm.x, h, l);
                    mrh[e] = h;
                    mrl[e] = l;
                    split_bf16(xm.y, h, l);
                    mih[e] = h;
                    mil[e] = l;
                }
                mma_split(aEr[n], arh, arl, jrh, jrl);
                mma_split(aEr[n], naih, nail, jih, jil);
                mma_split(aEr[n], nbrh, nbrl, mrh, mrl);
                mma_split(aEr[n], bih, bil, mih, mil);
                mma_split(aEi[n], arh, arl, jih, jil);
                mma_split(aEi[n], aih, ail, jrh, jrl);
                mma_split(aEi[n], nbrh, nbrl, mih, mil);
                mma_split(aEi[n], nbih, nbil, mrh, mrl);
                mma_split(aHr[n], drh, drl, jrh, jrl);
                mma_split(aHr[n], ndih, ndil, jih, jil);
                mma_split(aHr[n], crh, crl, mrh, mrl);
                mma_split(aHr[n], ncih, ncil, mih, mil);
                mma_split(aHi[n], drh, drl, jih, jil);
                mma_split(aHi[n], dih, dil, jrh, jrl);
                mma_split(aHi[n], crh, crl, mih, mil);
                mma_split(aHi[n], cih, cil, mrh, mrl);
            }
        }
    }
    if (wave > 0) {
#pragma unroll
        for (int n = 0; n < NT; ++n) {
            red[wave - 1][4 * n + 0][lane] = aEr[n];
            red[wave - 1][4 * n + 1][lane] = aEi[n];
            red[wave - 1][4 * n + 2][lane] = aHr[n];
            red[wave - 1][4 * n + 3][lane] = aHi[n];
        }
    }
    __syncthreads();
    if (wave != 0) return;
#pragma unroll
    for (int n = 0; n < NT; ++n) {
#pragma unroll
        for (int w = 0; w < MMA_WAVES - 1; ++w) {
            aEr[n] += red[w][4 * n + 0][lane];
            aEi[n] += red[w][4 * n + 1][lane];
            aHr[n] += red[w][4 * n + 2][lane];
            aHi[n] += red[w][4 * n + 3][lane];
        }
        const int rhs = 16 * n + lr;
        if (rhs >= R) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = row0 + 4 * lg + v;
            if (row >= nrow) continue;
            const int64_t iE = (int64_t)(2 * (r0 + row)) * R + rhs;
            const int64_t iH = iE + R;
            cx<float> qE = {aEr[n][v], aEi[n][v]}, qH = {aHr[n][v], aHi[n][v]};
            if (POLY) {
                if (dinv) edge_block(dinv + 4 * (int64_t)(r0 + row), qE, qH);
                cx<float> xe = x[iE], xh = x[iH];
                cx<float> ae = acc[iE], ah = acc[iH];
                cfma(ae, xe, inv_theta);
                cfma(ah, xh, inv_theta);
                acc[iE] = ae;
                acc[iH] = ah;
                if (write_y) {
                    cfms(xe, qE, inv_theta);
                    cfms(xh, qH, inv_theta);
                    y[iE] = xe;
                    y[iH] = xh;
                }
            } else {
                y[iE] = qE;
                y[iH] = qH;
            }
        }
    }
}


// Finest-level aggregation on the matrix cores (FP32):
//   S_t(k) += F_t(k) j + F_p(k) m,   S_p(k) += F_p(k) j - F_t(k) m,
// j = et s x_J, m = s x_M for the edges n of region box b.  Rows (M) are
// directions k, K runs over the box's edges, N over right-hand sides.  Grid
// (box, groups of 4 direction tiles); each wave owns one 16-direction tile.
template <int NT>
__global__ void __launch_bounds__(256) k_aggregate_mma(int K, int R, int nmt, const int *__restrict__ edge_ptr,
                                                       const int *__restrict__ edge_pos,
                                                       const int *__restrict__ edge_sign,
                                                       const cx<float> *__restrict__ tx, cx<float> et,
                                                       const cx<float> *__restrict__ x, cx<float> *__restrict__ S) {
    const int b = blockIdx.x;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int mt = blockIdx.y * 4 + wave;
    if (mt >= nmt) return;
    const int lr = lane & 15, lg = lane >> 4;
    const int e0 = edge_ptr[b], n = edge_ptr[b + 1] - e0;
    const int k = 16 * mt + lr;
    f32x4 tr[NT], ti[NT], pr[NT], pi[NT];
#pragma unroll
    for (int q = 0; q < NT; ++q) tr[q] = ti[q] = pr[q] = pi[q] = f32x4{0, 0, 0, 0};
    for (int s = 0; s < (n + 3) / 4; ++s) {
        const int e = 4 * s + lg;
        cx<float> ft = {0, 0}, fp = {0, 0};
        int p = -1;
        float sg = 0;
        if (e < n) {
            if (k < K) {
                ft = tx[(int64_t)(e0 + e) * 2 * K + k];
                fp = tx[(int64_t)(e0 + e) * 2 * K + K + k];
            }
            p = edge_pos[e0 + e];
            sg = (float)edge_sign[e0 + e];
        }
        const float nfti = -ft.y, nftr = -ft.x, nfpi = -fp.y;
#pragma unroll
        for (int q = 0; q < NT; ++q) {
            const int rhs = 16 * q + lr;
            cx<float> j = {0, 0}, m = {0, 0};
            if (p >= 0 && rhs < R) {
                const cx<float> xj = x[(int64_t)(2 * p) * R + rhs], xm = x[(int64_t)(2 * p + 1) * R + rhs];
                j = cmul(et, cx<float>{sg * xj.x, sg * xj.y});
                m = {sg * xm.x, sg * xm.y};
            }
            mma_f32(tr[q], ft.x, j.x);
            mma_f32(tr[q], nfti, j.y);
            mma_f32(tr[q], fp.x, m.x);
            mma_f32(tr[q], nfpi, m.y);
            mma_f32(ti[q], ft.x, j.y);
            mma_f32(ti[q], ft.y, j.x);
            mma_f32(ti[q], fp.x, m.y);
            mma_f32(ti[q], fp.y, m.x);
            mma_f32(pr[q], fp.x, j.x);
            mma_f32(pr[q], nfpi, j.y);
            mma_f32(pr[q], nftr, m.x);
            mma_f32(pr[q], ft.y, m.y);
            mma_f32(pi[q], fp.x, j.y);
            mma_f32(pi[q], fp.y, j.x);
            mma_f32(pi[q], nftr, m.y);
            mma_f32(pi[q], nfti, m.x);
        }
    }
    const int64_t KR = (int64_t)K * R;
#pragma unroll
    for (int q = 0; q < NT; ++q) {
        const int rhs = 16 * q + lr;
        if (rhs >= R) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int kk = 16 * mt + 4 * lg + v;
            if (kk >= K) continue;
            S[(int64_t)b * 2 * KR + (int64_t)kk * R + rhs] = {tr[q][v], ti[q][v]};
            S[(int64_t)b * 2 * KR + KR + (int64_t)kk * R + rhs] = {pr[q][v], pi[q][v]};
        }
    }
}

// Finest-level receive on the matrix cores (FP32):
//   y_E += s sum_k (R_t G_t + R_p G_p),  y_H += (s / et) sum_k (R_p G_t - R_t G_p)
// with R = conj(F) (real wavenumber) or the separate receive table.  Rows are
// the box's edges (16 per tile), K runs over directions (4 waves take every
// 4th step, partial sums added through LDS), N over right-hand sides.
// MODE 0 (PMCHWT) adds the sums as above.  JMCFIE / CNF run two passes:
// MODE 1 with the RWG table, y_E += c s R.G / et, y_H += c s R.(k x G)
// (c = tang, the weight of the tangential parts), and MODE 2 with the table
// of the rotated test functions N, y_E += N.(k x G) / et, y_H -= N.G.
template <int NT, bool LOSSY, int MODE>
__global__ void __launch_bounds__(64 * MMA_WAVES)
    k_receive_mma(int K, int R, const int *__restrict__ edge_ptr, const int *__restrict__ edge_pos,
                  const int *__restrict__ edge_sign, const cx<float> *__restrict__ tx,
                  const cx<float> *__restrict__ rx, cx<float> inv_et, float tang, const cx<float> *__restrict__ G,
                  cx<float> *__restrict__ y) {
    __shared__ f32x4 red[MMA_WAVES - 1][NT * 4][64];
    const int b = blockIdx.x, mt = blockIdx.y;
    const int e0 = edge_ptr[b], n = edge_ptr[b + 1] - e0;
    if (16 * mt >= n) return;   // uniform over the workgroup
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int lr = lane & 15, lg = lane >> 4;
    const int row = 16 * mt + lr;
    const cx<float> *tab = LOSSY ? rx : tx;
    const int64_t KR = (int64_t)K * R;
    const cx<float> *g = G + (int64_t)b * 2 * KR;
    f32x4 er[NT], ei[NT], hr[NT], hi[NT];
#pragma unroll
    for (int q = 0; q < NT; ++q) er[q] = ei[q] = hr[q] = hi[q] = f32x4{0, 0, 0, 0};
    for (int s = wave; s < (K + 3) / 4; s += MMA_WAVES) {
        const int k = 4 * s + lg;
        cx<float> rt = {0, 0}, rp = {0, 0};
        if (row < n && k < K) {
            rt = tab[(int64_t)(e0 + row) * 2 * K + k];
            rp = tab[(int64_t)(e0 + row) * 2 * K + K + k];
            if (!LOSSY) {
                rt.y = -rt.y;
                rp.y = -rp.y;
            }
        }
        const float nrti = -rt.y, nrtr = -rt.x, nrpi = -rp.y;
#pragma unroll
        for (int q = 0; q < NT; ++q) {
            const int rhs = 16 * q + lr;
            cx<float> gt = {0, 0}, gp = {0, 0};
            if (k < K && rhs < R) {
                gt = g[(int64_t)k * R + rhs];
                gp = g[KR + (int64_t)k * R + rhs];
            }
            mma_f32(er[q], rt.x, gt.x);
            mma_f32(er[q], nrti, gt.y);
            mma_f32(er[q], rp.x, gp.x);
            mma_f32(er[q], nrpi, gp.y);
            mma_f32(ei[q], rt.x, gt.y);
            mma_f32(ei[q], rt.y, gt.x);
            mma_f32(ei[q], rp.x, gp.y);
            mma_f32(ei[q], rp.y, gp.x);
            mma_f32(hr[q], nrtr, gp.x);
            mma_f32(hr[q], rt.y, gp.y);
            mma_f32(hr[q], rp.x, gt.x);
            mma_f32(hr[q], nrpi, gt.y);
            mma_f32(hi[q], nrtr, gp.y);
            mma_f32(hi[q], nrti, gp.x);
            mma_f32(hi[q], rp.x, gt.y);
            mma_f32(hi[q], rp.y, gt.x);
        }
    }
    if (wave > 0) {
#pragma unroll
        for (int q = 0; q < NT; ++q) {
            red[wave - 1][4 * q + 0][lane] = er[q];
            red[wave - 1][4 * q + 1][lane] = ei[q];
            red[wave - 1][4 * q + 2][lane] = hr[q];
            red[wave - 1][4 * q + 3][lane] = hi[q];
        }
    }
    __syncthreads();
    if (wave != 0) return;
#pragma unroll
    for (int q = 0; q < NT; ++q) {
#pragma unroll
        for (int w = 0; w < MMA_WAVES - 1; ++w) {
            er[q] += red[w][4 * q + 0][lane];
            ei[q] += red[w][4 * q + 1][lane];
            hr[q] += red[w][4 * q + 2][lane];
            hi[q] += red[w][4 * q + 3][lane];
        }
        const int rhs = 16 * q + lr;
        if (rhs >= R) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int ed = 16 * mt + 4 * lg + v;
            if (ed >= n) continue;
            const int p = edge_pos[e0 + ed];
            const float sg = (float)edge_sign[e0 + ed];
            const int64_t iE = (int64_t)(2 * p) * R + rhs, iH = iE + R;
            cx<float> ye = y[iE], yh = y[iH];
            if (MODE == 0) {
                const cx<float> hh = cmul(cx<float>{hr[q][v], hi[q][v]}, inv_et);
                ye.x += sg * er[q][v];
                ye.y += sg * ei[q][v];
                yh.x += sg * hh.x;
                yh.y += sg * hh.y;
            } else if (MODE == 1) {
                const float c = tang * sg;
                const cx<float> ee = cmul(cx<float>{c * er[q][v], c * ei[q][v]}, inv_et);
                ye.x += ee.x;
                ye.y += ee.y;
                yh.x += c * hr[q][v];
                yh.y += c * hi[q][v];
            } else {
                const cx<float> hh = cmul(cx<float>{hr[q][v], hi[q][v]}, inv_et);
                ye.x += hh.x;
                ye.y += hh.y;
                yh.x -= er[q][v];
                yh.y -= ei[q][v];
            }
            y[iE] = ye;
            y[iH] = yh;
        }
    }
}


// ---------------------------------------------------------------------------
// Interpolation (upward) and anterpolation (downward) on the matrix cores.
// The theta stage of a child pattern is, for every phi pair (j, j + h),
//   [T(:, j); T(:, j+h)] = W [f(:, j); f(:, j+h)],   W = [[A, B], [B, A]]
// (2 nth_p x 2 nth_c, real), and the phi stage with the child shift folded in
// is, for every parent theta row I, a complex matrix Dsh[slot][I] applied to
// T(I, :).  The intermediate T goes through HBM (tmp[c][comp][I][j][R]).
// Limits: 2 nth <= 64 and nph <= 64 (4 tiles of 16), checked by the host.
constexpr int IMT = 4;    // max 16-row tiles
constexpr int IKS = 16;   // max 4-column steps

// W (or its transpose) entry for the theta stage: row r, column k over
// [top/bottom half][theta index] blocks of sizes (nr, nk)
__device__ __forceinline__ float theta_w(const float *A, const float *B, int row, int col, int nr, int nk,
                                         int ldA, bool transpose) {
    if (row >= 2 * nr || col >= 2 * nk) return 0.f;
    const int hr = row >= nr, hc = col >= nk;
    const int r = row - hr * nr, c = col - hc * nk;
    // W[(hr, I)][(hc, i)] = A[I][i] if hr == hc else B[I][i]; transpose swaps roles
    const int I = transpose ? c : r, i = transpose ? r : c;
    return (hr == hc) ? A[I * ldA + i] : B[I * ldA + i];
}

// theta stage, upward: grid = children x 2 components.  W is staged in LDS in
// operand order; each wave takes (phi pair, 16-RHS tile) column blocks.
template <int NT>
__global__ void __launch_bounds__(256) k_up_theta_mma(int R, int nth_c, int nph_c, int nth_p,
                                                      const float *__restrict__ A, const float *__restrict__ B,
                                                      const cx<float> *__restrict__ Sc, cx<float> *__restrict__ tmp) {
    __shared__ float Wop[IMT * IKS * 64];
    const int c = blockIdx.x >> 1, comp = blockIdx.x & 1;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, lr = lane & 15, lg = lane >> 4;
    const int h = nph_c / 2, Kc = nth_c * nph_c;
    const int nmt = (2 * nth_p + 15) / 16, nks = (2 * nth_c + 3) / 4;
    for (int t = threadIdx.x; t < nmt * IKS * 64; t += 256) {   // only the row tiles in use are read
        const int l = t & 63, ms = t >> 6, mt = ms / IKS, st = ms % IKS;
        Wop[t] = theta_w(A, B, 16 * mt + (l & 15), 4 * st + (l >> 4), nth_p, nth_c, nth_c, false);
    }
    __syncthreads();
    const cx<float> *f = Sc + ((int64_t)c * 2 + comp) * Kc * R;
    cx<float> *out = tmp + ((int64_t)c * 2 + comp) * nth_p * nph_c * R;
    for (int ct = wave; ct < h * NT; ct += 4) {
        const int jp = ct / NT, n = ct % NT;
        const int rhs = 16 * n + lr;
        f32x4 re[IMT], im[IMT];
#pragma unroll
        for (int mt = 0; mt < IMT; ++mt) re[mt] = im[mt] = f32x4{0, 0, 0, 0};
        for (int st = 0; st < nks; ++st) {
            const int k = 4 * st + lg;
            const int hk = k >= nth_c, i = k - hk * nth_c;
            cx<float> fv = {0, 0};
            if (k < 2 * nth_c && rhs < R) fv = f[(int64_t)(i * nph_c + jp + hk * h) * R + rhs];
#pragma unroll
            for (int mt = 0; mt < IMT; ++mt) {
                if (mt < nmt) {
                    const float w = Wop[(mt * IKS + st) * 64 + lane];
                    mma_f32(re[mt], w, fv.x);
                    mma_f32(im[mt], w, fv.y);
                }
            }
        }
        if (rhs >= R) continue;
#pragma unroll
        for (int mt = 0; mt < IMT; ++mt) {
            if (mt >= nmt) continue;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = 16 * mt + 4 * lg + v;
                if (row >= 2 * nth_p) continue;
                const int hr = row >= nth_p, I = row - hr * nth_p;
                out[(int64_t)(I * nph_c + jp + hr * h) * R + rhs] = {re[mt][v], im[mt][v]};
            }
        }
    }
}

// phi stage + shift, upward: grid = parents x 2 x nth_p; wave w = 16-row
// tile of parent phi samples J; K runs over the children's phi samples, so
// the sum over children accumulates inside the matrix-core accumulators.
// Dsh[slot][I][J][j] = D[J][j] shift_up[slot][I nph_p + J] (complex).
// With one or two 16-row tiles of J per theta row, a workgroup takes
// mma_rows_per_wg(nph) theta rows (one per group of waves), so that all four
// waves work.
__host__ __device__ inline int mma_rows_per_wg(int nph) {
    const int ntl = (nph + 15) / 16;
    return ntl == 1 ? 4 : ntl == 2 ? 2 : 1;
}

template <int NT>
__global__ void __launch_bounds__(256) k_up_phi_mma(int R, int nth_p, int nph_p, int nph_c,
                                                    const cx<float> *__restrict__ Dsh,
                                                    const int *__restrict__ child_ptr,
                                                    const int *__restrict__ child_idx,
                                                    const int *__restrict__ child_slot,
                                                    const cx<float> *__restrict__ tmp, cx<float> *__restrict__ Sp) {
    const int ipb = mma_rows_per_wg(nph_p), nib = (nth_p + ipb - 1) / ipb, tpw = 4 / ipb;
    int bid = blockIdx.x;
    const int ib = bid % nib;
    bid /= nib;
    const int comp = bid % 2, P = bid / 2;
    const int wave0 = threadIdx.x >> 6, lane = threadIdx.x & 63, lr = lane & 15, lg = lane >> 4;
    const int wave = wave0 % tpw, I = ib * ipb + wave0 / tpw;   // tile of J, theta row
    if (16 * wave >= nph_p || I >= nth_p) return;
    const int J = 16 * wave + lr;
    f32x4 re[NT], im[NT];
#pragma unroll
    for (int n = 0; n < NT; ++n) re[n] = im[n] = f32x4{0, 0, 0, 0};
    for (int q = child_ptr[P]; q < child_ptr[P + 1]; ++q) {
        const int c = child_idx[q];
        const cx<float> *a_row = Dsh + (((int64_t)child_slot[c] * nth_p + I) * nph_p + J) * nph_c;
        const cx<float> *t = tmp + (((int64_t)c * 2 + comp) * nth_p + I) * nph_c * R;
        for (int st = 0; st < (nph_c + 3) / 4; ++st) {
            const int j = 4 * st + lg;
            cx<float> a = {0, 0};
            if (J < nph_p && j < nph_c) a = a_row[j];
            const float nay = -a.y;
#pragma unroll
            for (int n = 0; n < NT; ++n) {
                const int rhs = 16 * n + lr;
                cx<float> b = {0, 0};
                if (j < nph_c && rhs < R) b = t[(int64_t)j * R + rhs];
                mma_f32(re[n], a.x, b.x);
                mma_f32(re[n], nay, b.y);
                mma_f32(im[n], a.x, b.y);
                mma_f32(im[n], a.y, b.x);
            }
        }
    }
    cx<float> *out = Sp + (((int64_t)P * 2 + comp) * nth_p * nph_p + (int64_t)I * nph_p) * R;
#pragma unroll
    for (int n = 0; n < NT; ++n) {
        const int rhs = 16 * n + lr;
        if (rhs >= R) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int JJ = 16 * wave + 4 * lg + v;
            if (JJ < nph_p) out[(int64_t)JJ * R + rhs] = {re[n][v], im[n][v]};
        }
    }
}

// phi stage (transpose) + shift, downward: grid = children x 2 x nth_p;
// wave w = 16-row tile of child phi samples j; K runs over parent phi samples.
// Dsh[slot][I][j][J] = D[J][j] shift_dn[slot][I nph_p + J] (complex).
template <int NT>
__global__ void __launch_bounds__(256) k_dn_phi_mma(int R, int nth_p, int nph_p, int nph_c,
                                                    const cx<float> *__restrict__ Dsh,
                                                    const int *__restrict__ parent,
                                                    const int *__restrict__ child_slot,
                                                    const cx<float> *__restrict__ Gp, cx<float> *__restrict__ tmp) {
    const int ipb = mma_rows_per_wg(nph_c), nib = (nth_p + ipb - 1) / ipb, tpw = 4 / ipb;
    int bid = blockIdx.x;
    const int ib = bid % nib;
    bid /= nib;
    const int comp = bid % 2, c = bid / 2;
    const int wave0 = threadIdx.x >> 6, lane = threadIdx.x & 63, lr = lane & 15, lg = lane >> 4;
    const int wave = wave0 % tpw, I = ib * ipb + wave0 / tpw;   // tile of j, theta row
    if (16 * wave >= nph_c || I >= nth_p) return;
    const int j = 16 * wave + lr;
    const cx<float> *a_row = Dsh + (((int64_t)child_slot[c] * nth_p + I) * nph_c + j) * nph_p;
    const cx<float> *g = Gp + (((int64_t)parent[c] * 2 + comp) * nth_p * nph_p + (int64_t)I * nph_p) * R;
    f32x4 re[NT], im[NT];
#pragma unroll
    for (int n = 0; n < NT; ++n) re[n] = im[n] = f32x4{0, 0, 0, 0};
    for (int st = 0; st < (nph_p + 3) / 4; ++st) {
        const int J = 4 * st + lg;
        cx<float> a = {0, 0};
        if (j < nph_c && J < nph_p) a = a_row[J];
        const float nay = -a.y;
#pragma unroll
        for (int n = 0; n < NT; ++n) {
            const int rhs = 16 * n + lr;
            cx<float> b = {0, 0};
            if (J < nph_p && rhs < R) b = g[(int64_t)J * R + rhs];
            mma_f32(re[n], a.x, b.x);
            mma_f32(re[n], nay, b.y);
            mma_f32(im[n], a.x, b.y);
            mma_f32(im[n], a.y, b.x);
        }
    }
    cx<float> *out = tmp + (((int64_t)c * 2 + comp) * nth_p + I) * nph_c * R;
#pragma unroll
    for (int n = 0; n < NT; ++n) {
        const int rhs = 16 * n + lr;
        if (rhs >= R) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int jj = 16 * wave + 4 * lg + v;
            if (jj < nph_c) out[(int64_t)jj * R + rhs] = {re[n][v], im[n][v]};
        }
    }
}

// theta stage (transpose), downward: grid = children x 2; adds
// W^T [T(:, j); T(:, j+h)] into the child pattern (same blocking as upward).
template <int NT>
__global__ void __launch_bounds__(256) k_dn_theta_mma(int R, int nth_c, int nph_c, int nth_p,
                                                      const float *__restrict__ A, const float *__restrict__ B,
                                                      const cx<float> *__restrict__ tmp, cx<float> *__restrict__ Gc) {
    __shared__ float Wop[IMT * IKS * 64];
    const int c = blockIdx.x >> 1, comp = blockIdx.x & 1;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, lr = lane & 15, lg = lane >> 4;
    const int h = nph_c / 2, Kc = nth_c * nph_c;
    const int nmt = (2 * nth_c + 15) / 16, nks = (2 * nth_p + 3) / 4;
    for (int t = threadIdx.x; t < nmt * IKS * 64; t += 256) {   // only the row tiles in use are read
        const int l = t & 63, ms = t >> 6, mt = ms / IKS, st = ms % IKS;
        Wop[t] = theta_w(A, B, 16 * mt + (l & 15), 4 * st + (l >> 4), nth_c, nth_p, nth_c, true);
    }
    __syncthreads();
    const cx<float> *t = tmp + ((int64_t)c * 2 + comp) * nth_p * nph_c * R;
    cx<float> *out = Gc + ((int64_t)c * 2 + comp) * Kc * R;
    for (int ct = wave; ct < h * NT; ct += 4) {
        const int jp = ct / NT, n = ct % NT;
        const int rhs = 16 * n + lr;
        f32x4 re[IMT], im[IMT];
#pragma unroll
        for (int mt = 0; mt < IMT; ++mt) re[mt] = im[mt] = f32x4{0, 0, 0, 0};
        for (int st = 0; st < nks; ++st) {
            const int k = 4 * st + lg;
            const int hk = k >= nth_p, I = k - hk * nth_p;
            cx<float> tv = {0, 0};
            if (k < 2 * nth_p && rhs < R) tv = t[(int64_t)(I * nph_c + jp + hk * h) * R + rhs];
#pragma unroll
            for (int mt = 0; mt < IMT; ++mt) {
                if (mt < nmt) {
                    const float w = Wop[(mt * IKS + st) * 64 + lane];
                    mma_f32(re[mt], w, tv.x);
                    mma_f32(im[mt], w, tv.y);
                }
            }
        }
        if (rhs >= R) continue;
        // read all current values first, then add and store (no serialised
        // load-store chains)
        cx<float> cur[IMT][4];
#pragma unroll
        for (int mt = 0; mt < IMT; ++mt)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = 16 * mt + 4 * lg + v;
                cur[mt][v] = {0, 0};
                if (mt < nmt && row < 2 * nth_c) {
                    const int hr = row >= nth_c, i = row - hr * nth_c;
                    cur[mt][v] = out[(int64_t)(i * nph_c + jp + hr * h) * R + rhs];
                }
            }
#pragma unroll
        for (int mt = 0; mt < IMT; ++mt)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = 16 * mt + 4 * lg + v;
                if (mt < nmt && row < 2 * nth_c) {
                    const int hr = row >= nth_c, i = row - hr * nth_c;
                    out[(int64_t)(i * nph_c + jp + hr * h) * R + rhs] = {cur[mt][v].x + re[mt][v],
                                                                         cur[mt][v].y + im[mt][v]};
                }
            }
    }
}

}  // namespace sfmm
