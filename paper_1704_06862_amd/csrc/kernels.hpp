// gfx950 kernels of the MLFMM-accelerated PMCHWT product, its preconditioners
// and the batched FP64 Krylov solver.
//
// Internal layout (right-hand-side minor): position p of the internal edge
// order holds J_p and M~_p; unknown u = 2p + h (h = 0 for J, 1 for M~) of
// right-hand side r lives at index u * R + r.  Level patterns are
// [box][component][direction][r].  T is float or double; Krylov vectors are
// complex FP64 and right-hand-side major.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sfmm {

template <typename T>
struct alignas(2 * sizeof(T)) cx {
    T x, y;
};

template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ T fmad(T a, T b, T c) {
    if constexpr (sizeof(T) == 4) return __builtin_fmaf(a, b, c);
    else return __builtin_fma(a, b, c);
}
// acc += a b and acc -= a b as four fused multiply-adds
template <typename T>
__device__ __forceinline__ void cfma(cx<T> &acc, cx<T> a, cx<T> b) {
    acc.x = fmad(a.x, b.x, acc.x);
    acc.x = fmad(-a.y, b.y, acc.x);
    acc.y = fmad(a.x, b.y, acc.y);
    acc.y = fmad(a.y, b.x, acc.y);
}
template <typename T>
__device__ __forceinline__ void cfms(cx<T> &acc, cx<T> a, cx<T> b) {
    acc.x = fmad(-a.x, b.x, acc.x);
    acc.x = fmad(a.y, b.y, acc.x);
    acc.y = fmad(-a.x, b.y, acc.y);
    acc.y = fmad(-a.y, b.x, acc.y);
}
template <typename T>
__device__ __forceinline__ cx<T> cconj(cx<T> a) {
    return {a.x, -a.y};
}
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
// sum over the lanes that share lane % RT (the other lane bits)
template <int RT, typename T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
    for (int o = 32; o >= RT; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// (e, h) <- D (e, h) for one edge's 2x2 block d[0..3] (row-major)
template <typename T>
__device__ __forceinline__ void edge_block(const cx<T> *__restrict__ d, cx<T> &e, cx<T> &h) {
    const cx<T> d0 = d[0], d1 = d[1], d2 = d[2], d3 = d[3];
    cx<T> e2 = cmul(d0, e), h2 = cmul(d2, e);
    cfma(e2, d1, h);
    cfma(h2, d3, h);
    e = e2;
    h = h2;
}

constexpr int WG = 256;
constexpr int WAVES = WG / 64;
constexpr int RW = 8;               // rows (wavefronts) per near/ILU workgroup
constexpr int RWG = RW * 64;
constexpr int UPR = 4;              // parent theta rows per upward workgroup
constexpr int UPMAX = 8;            // outputs per thread in the upward kernel

// ---------------------------------------------------------------------------
// Layout conversions.

// boundary FP64 [R][J(ne); M~(ne)] -> internal T
template <typename T>
__global__ void k_to_internal(const double2 *__restrict__ xb, const int *__restrict__ pos, int ne, int R,
                              cx<T> *__restrict__ xi) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (int64_t)ne * R) return;
    const int e = (int)(id / R), r = (int)(id % R);
    const int p = pos[e];
    const double2 j = xb[(int64_t)r * 2 * ne + e], m = xb[(int64_t)r * 2 * ne + ne + e];
    xi[(int64_t)(2 * p) * R + r] = {(T)j.x, (T)j.y};
    xi[(int64_t)(2 * p + 1) * R + r] = {(T)m.x, (T)m.y};
}

template <typename T>
__global__ void k_to_boundary(const cx<T> *__restrict__ yi, const int *__restrict__ pos, int ne, int R,
                              double2 *__restrict__ yb) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (int64_t)ne * R) return;
    const int e = (int)(id / R), r = (int)(id % R);
    const int p = pos[e];
    const cx<T> j = yi[(int64_t)(2 * p) * R + r], m = yi[(int64_t)(2 * p + 1) * R + r];
    yb[(int64_t)r * 2 * ne + e] = make_double2((double)j.x, (double)j.y);
    yb[(int64_t)r * 2 * ne + ne + e] = make_double2((double)m.x, (double)m.y);
}

// Krylov FP64 vectors (slot s at base + act[s] * lds, internal order) <-> T [N][R]
template <typename T>
__global__ void k_gather(const double2 *__restrict__ base, int64_t lds, const int *__restrict__ act, int N, int R,
                         cx<T> *__restrict__ out) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (int64_t)N * R) return;
    const int i = (int)(id / R), s = (int)(id % R);
    const double2 v = base[(int64_t)act[s] * lds + i];
    out[id] = {(T)v.x, (T)v.y};
}

template <typename T>
__global__ void k_scatter(const cx<T> *__restrict__ in, int N, int R, const int *__restrict__ act, int64_t lds,
                          double2 *__restrict__ base) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (int64_t)N * R) return;
    const int i = (int)(id / R), s = (int)(id % R);
    const cx<T> v = in[id];
    base[(int64_t)act[s] * lds + i] = make_double2((double)v.x, (double)v.y);
}

// y = D x per edge (2x2 blocks dinv[4p..4p+3]) for R right-hand sides
template <typename T>
__global__ void k_edge_block(int ne, int R, const cx<T> *__restrict__ dinv, const cx<T> *__restrict__ x,
                             cx<T> *__restrict__ y) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (int64_t)ne * R) return;
    const int64_t p = id / R, r = id % R;
    cx<T> e = x[2 * p * R + r], h = x[(2 * p + 1) * R + r];
    edge_block(dinv + 4 * p, e, h);
    y[2 * p * R + r] = e;
    y[(2 * p + 1) * R + r] = h;
}

template <typename T>
__global__ void k_zero(cx<T> *__restrict__ a, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = {0, 0};
}

// ---------------------------------------------------------------------------
// Near-field product Y = Z_near X for a tile of RT right-hand sides.
// The box's input
// columns (both halves, RT right-hand sides) are staged in LDS; one wavefront
// per row; lane = rr + RT * cg (cg: column group), so the RT lanes of a
// column group share the matrix entries (one load serves RT products).
// POLY = true fuses one product-form step of the polynomial preconditioner:
// with Q = Z_near X,  acc += X / theta  and  Y = X - Q / theta.
template <typename T>
struct NearArgs {
    int R;
    const int *bstart, *col_ptr, *cols;
    const int64_t *val_ptr;
    const cx<T> *A, *B, *C, *x;
    cx<T> *y, *acc;
    cx<T> inv_theta;
    int write_y;
    const cx<T> *dinv;
    const cx<T> *D = nullptr;   // general block [[A, -B], [D, C]] (GEN kernels)
    // the same blocks rounded to bfloat16, (re, im) packed low/high in 32 bits
    // (H16 kernels: the polynomial preconditioner's products)
    const uint32_t *A16 = nullptr, *B16 = nullptr, *C16 = nullptr, *D16 = nullptr;
};

__device__ __forceinline__ cx<float> unpack_bf16x2(uint32_t u) {
    return cx<float>{__uint_as_float(u << 16), __uint_as_float(u & 0xffff0000u)};
}

// One workgroup of the near-field product: NRW rows (one wavefront each) of
// box b from row NRW * rg on, right-hand sides rhs0 .. rhs0 + RT - 1; xs is
// the LDS staging area of the box's input columns.
template <typename T, int RT, bool LDS, bool POLY, int NRW, bool GEN = false, bool H16 = false>
__device__ __forceinline__ void near_block(const NearArgs<T> &a, int b, int rg, int rhs0, cx<T> *xs) {
    static_assert(!H16 || std::is_same<T, float>::value, "bfloat16 blocks are read into FP32");
    constexpr int NCG = 64 / RT;
    const int r0 = a.bstart[b], nrow = a.bstart[b + 1] - r0;
    if (rg * NRW >= nrow) return;            // uniform over the workgroup
    const int c0 = a.col_ptr[b], ncol = a.col_ptr[b + 1] - c0;
    // LDS: the J inputs of all columns, then the M inputs ([2][ncol][RT]), so
    // that lanes reading consecutive columns touch consecutive 8-byte words
    if (LDS) {
        for (int t = threadIdx.x; t < ncol * 2 * RT; t += NRW * 64) {
            const int c = t / (2 * RT), hr = t % (2 * RT), h = hr / RT, r = hr % RT;
            const int p = a.cols[c0 + c];
            xs[(h * ncol + c) * RT + r] = a.x[(int64_t)(2 * p + h) * a.R + rhs0 + r];
        }
        __syncthreads();
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int row = rg * NRW + wave;
    if (row >= nrow) return;
    const int rr = lane % RT, cg = lane / RT;
    const int64_t rb = a.val_ptr[b] + (int64_t)row * ncol;
    auto xin = [&](int c, cx<T> &xj, cx<T> &xm) {
        if (LDS) {
            xj = xs[c * RT + rr];
            xm = xs[(ncol + c) * RT + rr];
        } else {
            const int p = a.cols[c0 + c];
            xj = a.x[(int64_t)(2 * p) * a.R + rhs0 + rr];
            xm = a.x[(int64_t)(2 * p + 1) * a.R + rhs0 + rr];
        }
    };
    // block entry i of plane P (FP32/FP64 or bfloat16 storage)
    auto ld = [&](const cx<T> *P, const uint32_t *P16, int64_t i) -> cx<T> {
        if constexpr (H16) {
            const cx<float> v = unpack_bf16x2(P16[i]);
            return cx<T>{v.x, v.y};
        } else {
            return P[i];
        }
    };
    cx<T> aE = {0, 0}, aH = {0, 0}, bE = {0, 0}, bH = {0, 0};
    int c = cg;
    for (; c + NCG < ncol; c += 2 * NCG) {
        const cx<T> a0 = ld(a.A, a.A16, rb + c), b0 = ld(a.B, a.B16, rb + c), c0v = ld(a.C, a.C16, rb + c);
        const cx<T> a1 = ld(a.A, a.A16, rb + c + NCG), b1 = ld(a.B, a.B16, rb + c + NCG),
                    c1v = ld(a.C, a.C16, rb + c + NCG);
        const cx<T> d0 = GEN ? ld(a.D, a.D16, rb + c) : b0, d1 = GEN ? ld(a.D, a.D16, rb + c + NCG) : b1;
        cx<T> xj0, xm0, xj1, xm1;
        xin(c, xj0, xm0);
        xin(c + NCG, xj1, xm1);
        cfma(aE, a0, xj0);
        cfms(aE, b0, xm0);
        cfma(aH, d0, xj0);
        cfma(aH, c0v, xm0);
        cfma(bE, a1, xj1);
        cfms(bE, b1, xm1);
        cfma(bH, d1, xj1);
        cfma(bH, c1v, xm1);
    }
    if (c < ncol) {
        const cx<T> a0 = ld(a.A, a.A16, rb + c), b0 = ld(a.B, a.B16, rb + c), c0v = ld(a.C, a.C16, rb + c);
        const cx<T> d0 = GEN ? ld(a.D, a.D16, rb + c) : b0;
        cx<T> xj0, xm0;
        xin(c, xj0, xm0);
        cfma(aE, a0, xj0);
        cfms(aE, b0, xm0);
        cfma(aH, d0, xj0);
        cfma(aH, c0v, xm0);
    }
    aE.x = group_sum<RT>(aE.x + bE.x);
    aE.y = group_sum<RT>(aE.y + bE.y);
    aH.x = group_sum<RT>(aH.x + bH.x);
    aH.y = group_sum<RT>(aH.y + bH.y);
    if (lane < RT) {
        const int64_t iE = (int64_t)(2 * (r0 + row)) * a.R + rhs0 + rr;
        const int64_t iH = iE + a.R;
        if (POLY) {
            cx<T> xe = a.x[iE], xh = a.x[iH];
            cx<T> ae = a.acc[iE], ah = a.acc[iH];
            cfma(ae, xe, a.inv_theta);
            cfma(ah, xh, a.inv_theta);
            a.acc[iE] = ae;
            a.acc[iH] = ah;
            if (a.write_y) {
                if (a.dinv) edge_block(a.dinv + 4 * (int64_t)(r0 + row), aE, aH);
                cfms(xe, aE, a.inv_theta);
                cfms(xh, aH, a.inv_theta);
                a.y[iE] = xe;
                a.y[iH] = xh;
            }
        } else {
            a.y[iE] = aE;
            a.y[iH] = aH;
        }
    }
}

// Grid: (finest boxes, row groups of RW rows, RHS tiles).  GEN: general
// blocks [[A, -B], [D, C]] (JMCFIE / CNF); otherwise D = B (PMCHWT).
// H16: the blocks are read from their bfloat16 copies A16 .. D16.
template <typename T, int RT, bool LDS, bool POLY, bool GEN, bool H16 = false>
__global__ void __launch_bounds__(RWG) k_near(int R, const int *__restrict__ bstart, const int *__restrict__ col_ptr,
                                              const int *__restrict__ cols, const int64_t *__restrict__ val_ptr,
                                              const cx<T> *__restrict__ A, const cx<T> *__restrict__ B,
                                              const cx<T> *__restrict__ C, const cx<T> *__restrict__ D,
                                              const cx<T> *__restrict__ x, cx<T> *__restrict__ y,
                                              cx<T> *__restrict__ acc, cx<T> inv_theta, int write_y,
                                              const cx<T> *__restrict__ dinv, const uint32_t *__restrict__ A16,
                                              const uint32_t *__restrict__ B16, const uint32_t *__restrict__ C16,
                                              const uint32_t *__restrict__ D16) {
    extern __shared__ unsigned char lds_raw[];
    NearArgs<T> a{R, bstart, col_ptr, cols, val_ptr, A, B, C, x, y, acc, inv_theta, write_y, dinv, D};
    a.A16 = A16;
    a.B16 = B16;
    a.C16 = C16;
    a.D16 = D16;
    near_block<T, RT, LDS, POLY, RW, GEN, H16>(a, (int)blockIdx.x, (int)blockIdx.y, (int)blockIdx.z * RT,
                                               reinterpret_cast<cx<T> *>(lds_raw));
}

// ---------------------------------------------------------------------------
// ILU(0) sweep over a range of boxes (one colour, or all boxes for the
// block-Jacobi variant): out_I = W_I [own_I ; other_K ...] for RT right-hand
// sides; grid = boxes x row groups x RHS tiles, one wavefront per unknown row.
template <typename T, int RT, bool LDS>
__global__ void __launch_bounds__(RWG) k_ilu(int R, int box0, const int *__restrict__ bstart,
                                             const int *__restrict__ col_ptr, const int *__restrict__ cols,
                                             const int64_t *__restrict__ val_ptr, const cx<T> *__restrict__ W,
                                             const cx<T> *__restrict__ own, const cx<T> *__restrict__ other,
                                             cx<T> *__restrict__ out) {
    extern __shared__ unsigned char lds_raw[];
    cx<T> *us = reinterpret_cast<cx<T> *>(lds_raw);     // [2 nc][RT]
    constexpr int NCG = 64 / RT;
    const int I = box0 + blockIdx.x;
    const int r0 = bstart[I], nI = bstart[I + 1] - r0;
    if ((int)blockIdx.y * RW >= 2 * nI) return;
    const int c0 = col_ptr[I], nc = col_ptr[I + 1] - c0;
    const int nu = 2 * nc;
    const int rhs0 = blockIdx.z * RT;
    auto src_of = [&](int t) { return (t < nI) ? own : other; };
    if (LDS) {
        for (int t = threadIdx.x; t < nu * RT; t += RWG) {
            const int cc = t / RT, rr = t % RT;
            const int e = cc >> 1;
            us[t] = src_of(e)[(int64_t)(2 * cols[c0 + e] + (cc & 1)) * R + rhs0 + rr];
        }
        __syncthreads();
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int row = blockIdx.y * RW + wave;
    if (row >= 2 * nI) return;
    const int rr = lane % RT, cg = lane / RT;
    const int64_t rb = val_ptr[I] + (int64_t)row * nu;
    auto uin = [&](int cc) -> cx<T> {
        if (LDS) return us[cc * RT + rr];
        const int e = cc >> 1;
        return src_of(e)[(int64_t)(2 * cols[c0 + e] + (cc & 1)) * R + rhs0 + rr];
    };
    cx<T> a0 = {0, 0}, a1 = {0, 0};
    int cc = cg;
    for (; cc + NCG < nu; cc += 2 * NCG) {
        cfma(a0, W[rb + cc], uin(cc));
        cfma(a1, W[rb + cc + NCG], uin(cc + NCG));
    }
    if (cc < nu) cfma(a0, W[rb + cc], uin(cc));
    a0.x = group_sum<RT>(a0.x + a1.x);
    a0.y = group_sum<RT>(a0.y + a1.y);
    if (lane < RT) out[(int64_t)(2 * r0 + row) * R + rhs0 + rr] = a0;
}

// ---------------------------------------------------------------------------
// Finest-level aggregation: S_b[c][k][r] = sum_n s_n (...)(theta, phi).
// One workgroup per region box; threads over (direction, rhs) with rhs
// fastest, so the R threads of a direction share each pattern load; the
// box's scaled excitations are staged in LDS in chunks of ech edges.
template <typename T>
struct AggRegion {
    int K, nbf;                          // directions, region boxes
    const int *edge_ptr, *edge_pos, *edge_sign;
    const cx<T> *tx;
    cx<T> et;
    cx<T> *S;
};

template <typename T>
__device__ __forceinline__ void aggregate_box(int K, int R, int ech, const int *__restrict__ edge_ptr,
                                              const int *__restrict__ edge_pos, const int *__restrict__ edge_sign,
                                              const cx<T> *__restrict__ tx, cx<T> et, const cx<T> *__restrict__ x,
                                              cx<T> *__restrict__ S, int b);

// Up to two regions per launch: workgroups 0 .. r0.nbf - 1 take region r0's
// boxes, the next r1.nbf those of r1.
template <typename T>
__global__ void __launch_bounds__(1024) k_aggregate(const AggRegion<T> r0, const AggRegion<T> r1, int R, int ech,
                                                    const cx<T> *__restrict__ x) {
    const bool second = (int)blockIdx.x >= r0.nbf;
    const AggRegion<T> &rg = second ? r1 : r0;
    const int b = second ? (int)blockIdx.x - r0.nbf : (int)blockIdx.x;
    aggregate_box<T>(rg.K, R, ech, rg.edge_ptr, rg.edge_pos, rg.edge_sign, rg.tx, rg.et, x, rg.S, b);
}

template <typename T>
__device__ __forceinline__ void aggregate_box(int K, int R, int ech, const int *__restrict__ edge_ptr,
                                              const int *__restrict__ edge_pos, const int *__restrict__ edge_sign,
                                              const cx<T> *__restrict__ tx, cx<T> et, const cx<T> *__restrict__ x,
                                              cx<T> *__restrict__ S, int b) {
    extern __shared__ unsigned char lds_raw[];
    cx<T> *js = reinterpret_cast<cx<T> *>(lds_raw);      // [ech][R]
    cx<T> *ms = js + (size_t)ech * R;
    const int e0 = edge_ptr[b], e1 = edge_ptr[b + 1];
    const int KR = K * R;
    for (int q0 = 0; q0 < KR; q0 += blockDim.x) {
        const int q = q0 + threadIdx.x;
        const int k = q / R, r = q % R;
        cx<T> st = {0, 0}, sp = {0, 0}, st2 = {0, 0}, sp2 = {0, 0};
        for (int c0 = e0; c0 < e1; c0 += ech) {
            const int cnt = min(ech, e1 - c0);
            __syncthreads();
            for (int t = threadIdx.x; t < cnt * R; t += blockDim.x) {
                const int te = t / R, tr = t % R;
                const int p = edge_pos[c0 + te];
                const T s = (T)edge_sign[c0 + te];
                const cx<T> xj = x[(int64_t)(2 * p) * R + tr], xm = x[(int64_t)(2 * p + 1) * R + tr];
                const cx<T> j = cmul(et, xj);
                js[t] = {s * j.x, s * j.y};
                ms[t] = {s * xm.x, s * xm.y};
            }
            __syncthreads();
            if (q < KR) {
                const cx<T> *F = tx + (size_t)c0 * 2 * K + k;
                int t = 0;
                for (; t + 3 < cnt; t += 4) {
                    const cx<T> ft = F[(size_t)t * 2 * K], fp = F[(size_t)t * 2 * K + K];
                    const cx<T> gt = F[(size_t)(t + 1) * 2 * K], gp = F[(size_t)(t + 1) * 2 * K + K];
                    const cx<T> ut = F[(size_t)(t + 2) * 2 * K], up = F[(size_t)(t + 2) * 2 * K + K];
                    const cx<T> vt = F[(size_t)(t + 3) * 2 * K], vp = F[(size_t)(t + 3) * 2 * K + K];
                    const cx<T> j0 = js[t * R + r], m0 = ms[t * R + r];
                    const cx<T> j1 = js[(t + 1) * R + r], m1 = ms[(t + 1) * R + r];
                    const cx<T> j2 = js[(t + 2) * R + r], m2 = ms[(t + 2) * R + r];
                    const cx<T> j3 = js[(t + 3) * R + r], m3 = ms[(t + 3) * R + r];
                    cfma(st, ft, j0);
                    cfma(st, fp, m0);
                    cfma(sp, fp, j0);
                    cfms(sp, ft, m0);
                    cfma(st2, gt, j1);
                    cfma(st2, gp, m1);
                    cfma(sp2, gp, j1);
                    cfms(sp2, gt, m1);
                    cfma(st, ut, j2);
                    cfma(st, up, m2);
                    cfma(sp, up, j2);
                    cfms(sp, ut, m2);
                    cfma(st2, vt, j3);
                    cfma(st2, vp, m3);
                    cfma(sp2, vp, j3);
                    cfms(sp2, vt, m3);
                }
                for (; t + 1 < cnt; t += 2) {
                    const cx<T> ft = F[(size_t)t * 2 * K], fp = F[(size_t)t * 2 * K + K];
                    const cx<T> gt = F[(size_t)(t + 1) * 2 * K], gp = F[(size_t)(t + 1) * 2 * K + K];
                    const cx<T> j0 = js[t * R + r], m0 = ms[t * R + r];
                    const cx<T> j1 = js[(t + 1) * R + r], m1 = ms[(t + 1) * R + r];
                    cfma(st, ft, j0);
                    cfma(st, fp, m0);
                    cfma(sp, fp, j0);
                    cfms(sp, ft, m0);
                    cfma(st2, gt, j1);
                    cfma(st2, gp, m1);
                    cfma(sp2, gp, j1);
                    cfms(sp2, gt, m1);
                }
                if (t < cnt) {
                    const cx<T> ft = F[(size_t)t * 2 * K], fp = F[(size_t)t * 2 * K + K];
                    const cx<T> j0 = js[t * R + r], m0 = ms[t * R + r];
                    cfma(st, ft, j0);
                    cfma(st, fp, m0);
                    cfma(sp, fp, j0);
                    cfms(sp, ft, m0);
                }
            }
        }
        if (q < KR) {
            S[((size_t)b * 2 * K + k) * R + r] = {st.x + st2.x, st.y + st2.y};
            S[((size_t)b * 2 * K + K + k) * R + r] = {sp.x + sp2.x, sp.y + sp2.y};
        }
    }
}

// ---------------------------------------------------------------------------
// Upward pass.  One workgroup per (parent box, component, chunk of UPR parent
// theta rows, tile of RT right-hand sides): for every child in turn its
// pattern is staged in LDS, the theta stage computes the chunk's rows into LDS
// (even/odd azimuthal parts paired through phi and phi + pi), and the phi
// stage (transposed matrix, coalesced) plus the child shift accumulates the
// chunk's outputs in registers.
template <typename T, int RT>
__global__ void __launch_bounds__(WG) k_up_box(int R, int nth_c, int nph_c, int nth_p, int nph_p,
                                               const T *__restrict__ A, const T *__restrict__ B,
                                               const T *__restrict__ Dt, const int *__restrict__ child_ptr,
                                               const int *__restrict__ child_idx, const int *__restrict__ child_slot,
                                               const cx<T> *__restrict__ shift, const cx<T> *__restrict__ Sc,
                                               cx<T> *__restrict__ Sp) {
    extern __shared__ unsigned char lds_raw[];
    const int Kc = nth_c * nph_c, Kp = nth_p * nph_p;
    cx<T> *fs = reinterpret_cast<cx<T> *>(lds_raw);      // [Kc][RT]
    cx<T> *ts = fs + (size_t)Kc * RT;                     // [UPR][nph_c][RT]
    const int nchunk = (nth_p + UPR - 1) / UPR;
    const int ntile = R / RT;
    int bid = blockIdx.x;
    const int tile = bid % ntile;
    bid /= ntile;
    const int chunk = bid % nchunk;
    bid /= nchunk;
    const int comp = bid % 2;
    const int P = bid / 2;
    const int I0 = chunk * UPR;
    const int nI = min(UPR, nth_p - I0);
    const int nout = nI * nph_p * RT;
    const int h = nph_c / 2;
    const int rhs0 = tile * RT;
    cx<T> acc[UPMAX];
#pragma unroll
    for (int u = 0; u < UPMAX; ++u) acc[u] = {0, 0};
    for (int q = child_ptr[P]; q < child_ptr[P + 1]; ++q) {
        const int c = child_idx[q];
        const cx<T> *f = Sc + ((size_t)c * 2 + comp) * Kc * R;
        __syncthreads();
        for (int t = threadIdx.x; t < Kc * RT; t += WG) fs[t] = f[(size_t)(t / RT) * R + rhs0 + t % RT];
        __syncthreads();
        for (int t = threadIdx.x; t < nI * nph_c * RT; t += WG) {
            const int rr = t % RT, tj = t / RT;
            const int I = I0 + tj / nph_c, j = tj % nph_c;
            const int j1 = j < h ? j : j - h, j2 = j1 + h;
            const T *Pa = (j < h) ? A : B;
            const T *Pb = (j < h) ? B : A;
            cx<T> a2 = {0, 0};
            for (int i = 0; i < nth_c; ++i) {
                const T a = Pa[I * nth_c + i], b = Pb[I * nth_c + i];
                const cx<T> f1 = fs[(i * nph_c + j1) * RT + rr], f2 = fs[(i * nph_c + j2) * RT + rr];
                a2.x += a * f1.x + b * f2.x;
                a2.y += a * f1.y + b * f2.y;
            }
            ts[t] = a2;
        }
        __syncthreads();
        const cx<T> *sh = shift + (size_t)child_slot[c] * Kp + I0 * nph_p;
#pragma unroll
        for (int u = 0; u < UPMAX; ++u) {
            const int o = threadIdx.x + u * WG;
            if (o < nout) {
                const int rr = o % RT, oj = o / RT;
                const int Il = oj / nph_p, J = oj % nph_p;
                const cx<T> *g = ts + (size_t)Il * nph_c * RT + rr;
                cx<T> v = {0, 0};
                for (int j = 0; j < nph_c; ++j) {
                    const T d = Dt[(size_t)j * nph_p + J];
                    v.x += d * g[j * RT].x;
                    v.y += d * g[j * RT].y;
                }
                cfma(acc[u], sh[oj], v);
            }
        }
    }
    cx<T> *out = Sp + (((size_t)P * 2 + comp) * Kp + I0 * nph_p) * R + rhs0;
#pragma unroll
    for (int u = 0; u < UPMAX; ++u) {
        const int o = threadIdx.x + u * WG;
        if (o < nout) out[(size_t)(o / RT) * R + o % RT] = acc[u];
    }
}

// Downward pass (transpose of the upward pass), one workgroup per (child box,
// RHS tile): shifted parent pattern -> LDS, phi transpose -> LDS, theta
// transpose accumulated into the child pattern.
template <typename T, int RT>
__global__ void __launch_bounds__(WG) k_dn_box(int R, int nth_c, int nph_c, int nth_p, int nph_p,
                                               const T *__restrict__ A, const T *__restrict__ B,
                                               const T *__restrict__ D, const int *__restrict__ parent,
                                               const int *__restrict__ child_slot, const cx<T> *__restrict__ shift,
                                               const cx<T> *__restrict__ Gp, cx<T> *__restrict__ Gc) {
    extern __shared__ unsigned char lds_raw[];
    const int Kc = nth_c * nph_c, Kp = nth_p * nph_p;
    cx<T> *gs = reinterpret_cast<cx<T> *>(lds_raw);      // [Kp][RT]
    cx<T> *ts = gs + (size_t)Kp * RT;                     // [nth_p][nph_c][RT]
    const int ntile = R / RT;
    const int c = blockIdx.x / ntile, tile = blockIdx.x % ntile;
    const int rhs0 = tile * RT;
    const int h = nph_c / 2;
    const cx<T> *sh = shift + (size_t)child_slot[c] * Kp;
    for (int comp = 0; comp < 2; ++comp) {
        const cx<T> *g = Gp + ((size_t)parent[c] * 2 + comp) * Kp * R;
        __syncthreads();
        for (int t = threadIdx.x; t < Kp * RT; t += WG)
            gs[t] = cmul(sh[t / RT], g[(size_t)(t / RT) * R + rhs0 + t % RT]);
        __syncthreads();
        for (int t = threadIdx.x; t < nth_p * nph_c * RT; t += WG) {
            const int rr = t % RT, tj = t / RT;
            const int I = tj / nph_c, j = tj % nph_c;
            const cx<T> *row = gs + (size_t)I * nph_p * RT + rr;
            cx<T> a2 = {0, 0};
            for (int J = 0; J < nph_p; ++J) {
                const T d = D[(size_t)J * nph_c + j];
                a2.x += d * row[J * RT].x;
                a2.y += d * row[J * RT].y;
            }
            ts[t] = a2;
        }
        __syncthreads();
        cx<T> *out = Gc + ((size_t)c * 2 + comp) * Kc * R + rhs0;
        for (int t = threadIdx.x; t < Kc * RT; t += WG) {
            const int rr = t % RT, tk = t / RT;
            const int i = tk / nph_c, j = tk % nph_c;
            const int j1 = j < h ? j : j - h, j2 = j1 + h;
            const T *Pa = (j < h) ? A : B;
            const T *Pb = (j < h) ? B : A;
            cx<T> a2 = out[(size_t)tk * R + rr];
            for (int I = 0; I < nth_p; ++I) {
                const T a = Pa[I * nth_c + i], b = Pb[I * nth_c + i];
                const cx<T> g1 = ts[(I * nph_c + j1) * RT + rr], g2 = ts[(I * nph_c + j2) * RT + rr];
                a2.x += a * g1.x + b * g2.x;
                a2.y += a * g1.y + b * g2.y;
            }
            out[(size_t)tk * R + rr] = a2;
        }
    }
}

// Element-wise fallbacks for levels whose box patterns exceed the LDS budget.
// theta stage: tmp[c][comp][I][j][r]
template <typename T>
__global__ void k_up_theta(int R, int nchild, int nth_c, int nph_c, int nth_p, const T *__restrict__ A,
                           const T *__restrict__ B, const cx<T> *__restrict__ S, cx<T> *__restrict__ tmp) {
    const int64_t total = (int64_t)nchild * 2 * nth_p * nph_c * R;
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= total) return;
    const int r = id % R;
    int64_t q = id / R;
    const int j = q % nph_c;
    q /= nph_c;
    const int I = q % nth_p;
    const int64_t cc = q / nth_p;
    const int h = nph_c / 2;
    const int j1 = j < h ? j : j - h, j2 = j1 + h;
    const T *Pa = (j < h) ? A : B;
    const T *Pb = (j < h) ? B : A;
    const cx<T> *f = S + cc * nth_c * nph_c * R + r;
    cx<T> acc = {0, 0};
    for (int i = 0; i < nth_c; ++i) {
        const T a = Pa[I * nth_c + i], b = Pb[I * nth_c + i];
        const cx<T> f1 = f[(size_t)(i * nph_c + j1) * R], f2 = f[(size_t)(i * nph_c + j2) * R];
        acc.x += a * f1.x + b * f2.x;
        acc.y += a * f1.y + b * f2.y;
    }
    tmp[id] = acc;
}

// phi stage + shift + sum over the children of every parent
template <typename T>
__global__ void k_up_phi(int R, int nparent, int nth_p, int nph_p, int nph_c, const T *__restrict__ Dt,
                         const int *__restrict__ child_ptr, const int *__restrict__ child_idx,
                         const int *__restrict__ child_slot, const cx<T> *__restrict__ shift,
                         const cx<T> *__restrict__ tmp, cx<T> *__restrict__ Sp) {
    const int Kp = nth_p * nph_p;
    const int64_t total = (int64_t)nparent * 2 * Kp * R;
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= total) return;
    const int r = id % R;
    int64_t q = id / R;
    const int kk = q % Kp;
    q /= Kp;
    const int comp = q % 2;
    const int P = q / 2;
    const int I = kk / nph_p, J = kk % nph_p;
    cx<T> out = {0, 0};
    for (int qq = child_ptr[P]; qq < child_ptr[P + 1]; ++qq) {
        const int c = child_idx[qq];
        const cx<T> *g = tmp + ((((int64_t)c * 2 + comp) * nth_p + I) * nph_c) * R + r;
        cx<T> v = {0, 0};
        for (int j = 0; j < nph_c; ++j) {
            const T d = Dt[(size_t)j * nph_p + J];
            v.x += d * g[(size_t)j * R].x;
            v.y += d * g[(size_t)j * R].y;
        }
        cfma(out, shift[child_slot[c] * Kp + kk], v);
    }
    Sp[id] = out;
}

// downward phi stage: tmp[c][comp][I][j][r] = sum_J D[J][j] shift_dn G_parent
template <typename T>
__global__ void k_dn_phi(int R, int nchild, int nth_p, int nph_p, int nph_c, const T *__restrict__ D,
                         const int *__restrict__ parent, const int *__restrict__ child_slot,
                         const cx<T> *__restrict__ shift, const cx<T> *__restrict__ Gp, cx<T> *__restrict__ tmp) {
    const int Kp = nth_p * nph_p;
    const int64_t total = (int64_t)nchild * 2 * nth_p * nph_c * R;
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= total) return;
    const int r = id % R;
    int64_t q = id / R;
    const int j = q % nph_c;
    q /= nph_c;
    const int I = q % nth_p;
    q /= nth_p;
    const int comp = q % 2;
    const int c = q / 2;
    const cx<T> *g = Gp + (((int64_t)parent[c] * 2 + comp) * Kp + I * nph_p) * R + r;
    const cx<T> *sh = shift + child_slot[c] * Kp + I * nph_p;
    cx<T> acc = {0, 0};
    for (int J = 0; J < nph_p; ++J) {
        const cx<T> v = cmul(sh[J], g[(size_t)J * R]);
        const T d = D[J * nph_c + j];
        acc.x += d * v.x;
        acc.y += d * v.y;
    }
    tmp[id] = acc;
}

// downward theta stage, accumulated into G_child[c][comp][i][j][r]
template <typename T>
__global__ void k_dn_theta(int R, int nchild, int nth_c, int nph_c, int nth_p, const T *__restrict__ A,
                           const T *__restrict__ B, const cx<T> *__restrict__ tmp, cx<T> *__restrict__ Gc) {
    const int64_t total = (int64_t)nchild * 2 * nth_c * nph_c * R;
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= total) return;
    const int r = id % R;
    int64_t q = id / R;
    const int j = q % nph_c;
    q /= nph_c;
    const int i = q % nth_c;
    const int64_t cc = q / nth_c;
    const int h = nph_c / 2;
    const int j1 = j < h ? j : j - h, j2 = j1 + h;
    const T *Pa = (j < h) ? A : B;
    const T *Pb = (j < h) ? B : A;
    const cx<T> *g = tmp + cc * nth_p * nph_c * R + r;
    cx<T> acc = Gc[id];
    for (int I = 0; I < nth_p; ++I) {
        const T a = Pa[I * nth_c + i], b = Pb[I * nth_c + i];
        const cx<T> g1 = g[(size_t)(I * nph_c + j1) * R], g2 = g[(size_t)(I * nph_c + j2) * R];
        acc.x += a * g1.x + b * g2.x;
        acc.y += a * g1.y + b * g2.y;
    }
    Gc[id] = acc;
}

// ---------------------------------------------------------------------------
// One right-hand side: the same two stages as the element-wise kernels above,
// register-blocked, with the interpolation matrices staged in LDS, and one
// launch for the same level transition of every region (a list of up to
// SPLIT_MAXJOB jobs; the workgroups [blk0[i], blk0[i + 1]) serve job i).  In
// the theta stages a thread computes two theta rows by the azimuthal pair
// (j, j + h), h = nph_c / 2 (the two halves of the paired matrix
// [[A, B], [B, A]] share every load); in the phi stages a thread computes two
// adjacent azimuths of one theta row.  BS threads per workgroup: transitions
// with few items use 64 so the workgroups spread evenly over the CUs.
constexpr int SPLIT_MAXJOB = 8;

template <typename P>
struct JobList {
    int n;
    int blk0[SPLIT_MAXJOB + 1];
    P p[SPLIT_MAXJOB];
};

// the job of this workgroup (workgroup-uniform) and the workgroup's index in it
template <typename P>
__device__ __forceinline__ const P &job_at(const JobList<P> &jl, int blk, int &local) {
    int i = 0;
    while (i + 1 < jl.n && blk >= jl.blk0[i + 1]) ++i;
    local = blk - jl.blk0[i];
    return jl.p[i];
}
template <typename P>
__device__ __forceinline__ const P &job_of(const JobList<P> &jl, int &local) {
    return job_at(jl, (int)blockIdx.x, local);
}

template <typename T>
struct ThetaJob {   // up: tmp[cc][I][j] from S[cc][i][j]; down: Gc[cc][i][j] += from tmp[cc][I][j]
    int ncc, nth_c, nph_c, nth_p;
    const T *A, *B;
    const cx<T> *in;
    cx<T> *out;
};
template <typename T>
struct UpPhiJob {
    int nparent, nth_p, nph_p, nph_c;
    const T *Dt;
    const int *child_ptr, *child_idx, *child_slot;
    const cx<T> *shift, *tmp;
    cx<T> *Sp;
};
template <typename T>
struct DnPhiJob {
    int nchild, nth_p, nph_p, nph_c;
    const T *D;
    const int *parent, *child_slot;
    const cx<T> *shift, *Gp;
    cx<T> *tmp;
};

// tmp[cc][I][j] = sum_i A/B[I][i] S[cc][i][j or j +- h], cc = 2 child + comp
template <typename T, int BS>
__global__ void __launch_bounds__(BS) k_up_theta1(const JobList<ThetaJob<T>> jl) {
    extern __shared__ unsigned char lds_raw[];
    int local;
    const ThetaJob<T> &a = job_of(jl, local);
    const int nth_c = a.nth_c, nph_c = a.nph_c, nth_p = a.nth_p;
    T *As = reinterpret_cast<T *>(lds_raw);   // [nth_p][nth_c]
    T *Bs = As + nth_p * nth_c;
    for (int t = threadIdx.x; t < nth_p * nth_c; t += BS) {
        As[t] = a.A[t];
        Bs[t] = a.B[t];
    }
    __syncthreads();
    const int h = nph_c / 2, np2 = (nth_p + 1) / 2;
    const int id = local * BS + (int)threadIdx.x;   // item counts fit in 32 bits (checked by the host)
    if (id >= a.ncc * np2 * h) return;
    const int j = id % h;
    const int I = 2 * ((id / h) % np2);
    const int64_t cc = id / (h * np2);
    const bool two = I + 1 < nth_p;
    const int I1 = two ? I + 1 : I;
    const cx<T> *f = a.in + cc * nth_c * nph_c;
    cx<T> a0 = {0, 0}, a1 = {0, 0}, b0 = {0, 0}, b1 = {0, 0};   // rows I, I1; azimuths j, j + h
    for (int i = 0; i < nth_c; ++i) {
        const T p0 = As[I * nth_c + i], q0 = Bs[I * nth_c + i];
        const T p1 = As[I1 * nth_c + i], q1 = Bs[I1 * nth_c + i];
        const cx<T> f1 = f[i * nph_c + j], f2 = f[i * nph_c + j + h];
        a0.x += p0 * f1.x + q0 * f2.x;
        a0.y += p0 * f1.y + q0 * f2.y;
        b0.x += q0 * f1.x + p0 * f2.x;
        b0.y += q0 * f1.y + p0 * f2.y;
        a1.x += p1 * f1.x + q1 * f2.x;
        a1.y += p1 * f1.y + q1 * f2.y;
        b1.x += q1 * f1.x + p1 * f2.x;
        b1.y += q1 * f1.y + p1 * f2.y;
    }
    cx<T> *o = a.out + (cc * nth_p + I) * nph_c;
    o[j] = a0;
    o[j + h] = b0;
    if (two) {
        o[nph_c + j] = a1;
        o[nph_c + j + h] = b1;
    }
}

// Sp[P][comp][I][J] = sum_children shift[slot][I][J] sum_j Dt[j][J] tmp[c][comp][I][j]
template <typename T, int BS>
__device__ __forceinline__ void up_phi1_block(const JobList<UpPhiJob<T>> &jl, int blk, unsigned char *lds_raw) {
    int local;
    const UpPhiJob<T> &a = job_at(jl, blk, local);
    const int nth_p = a.nth_p, nph_p = a.nph_p, nph_c = a.nph_c;
    T *Ds = reinterpret_cast<T *>(lds_raw);   // [nph_c][nph_p]
    for (int t = threadIdx.x; t < nph_c * nph_p; t += BS) Ds[t] = a.Dt[t];
    __syncthreads();
    const int Kp = nth_p * nph_p, hp = nph_p / 2;
    const int id = local * BS + (int)threadIdx.x;
    if (id >= a.nparent * 2 * nth_p * hp) return;
    const int J = 2 * (id % hp);
    int q = id / hp;
    const int I = q % nth_p;
    q /= nth_p;
    const int comp = q % 2;
    const int P = q / 2;
    cx<T> o0 = {0, 0}, o1 = {0, 0};
    for (int qq = a.child_ptr[P]; qq < a.child_ptr[P + 1]; ++qq) {
        const int c = a.child_idx[qq];
        const cx<T> *g = a.tmp + (((int64_t)c * 2 + comp) * nth_p + I) * nph_c;
        cx<T> v0 = {0, 0}, v1 = {0, 0};
        for (int j = 0; j < nph_c; ++j) {
            // one paired LDS read of (J, J + 1): J and nph_p are even
            const cx<T> dd = *reinterpret_cast<const cx<T> *>(Ds + j * nph_p + J);
            const T d0 = dd.x, d1 = dd.y;
            const cx<T> t = g[j];
            v0.x += d0 * t.x;
            v0.y += d0 * t.y;
            v1.x += d1 * t.x;
            v1.y += d1 * t.y;
        }
        const cx<T> *sh = a.shift + (size_t)a.child_slot[c] * Kp + I * nph_p + J;
        cfma(o0, sh[0], v0);
        cfma(o1, sh[1], v1);
    }
    cx<T> *out = a.Sp + ((int64_t)P * 2 + comp) * Kp + I * nph_p + J;
    out[0] = o0;
    out[1] = o1;
}

template <typename T, int BS>
__global__ void __launch_bounds__(BS) k_up_phi1(const JobList<UpPhiJob<T>> jl) {
    extern __shared__ unsigned char lds_raw[];
    up_phi1_block<T, BS>(jl, (int)blockIdx.x, lds_raw);
}

// tmp[c][comp][I][j] = sum_J D[J][j] shift_dn[slot][I][J] Gp[parent][comp][I][J]
template <typename T, int BS>
__global__ void __launch_bounds__(BS) k_dn_phi1(const JobList<DnPhiJob<T>> jl) {
    extern __shared__ unsigned char lds_raw[];
    int local;
    const DnPhiJob<T> &a = job_of(jl, local);
    const int nth_p = a.nth_p, nph_p = a.nph_p, nph_c = a.nph_c;
    T *Ds = reinterpret_cast<T *>(lds_raw);   // [nph_p][nph_c]
    for (int t = threadIdx.x; t < nph_p * nph_c; t += BS) Ds[t] = a.D[t];
    __syncthreads();
    const int Kp = nth_p * nph_p, hc = nph_c / 2;
    const int id = local * BS + (int)threadIdx.x;
    if (id >= a.nchild * 2 * nth_p * hc) return;
    const int j = 2 * (id % hc);
    int q = id / hc;
    const int I = q % nth_p;
    q /= nth_p;
    const int comp = q % 2;
    const int c = q / 2;
    const cx<T> *g = a.Gp + ((int64_t)a.parent[c] * 2 + comp) * Kp + I * nph_p;
    const cx<T> *sh = a.shift + (size_t)a.child_slot[c] * Kp + I * nph_p;
    cx<T> a0 = {0, 0}, a1 = {0, 0};
    for (int J = 0; J < nph_p; ++J) {
        const cx<T> v = cmul(sh[J], g[J]);
        const T d0 = Ds[J * nph_c + j], d1 = Ds[J * nph_c + j + 1];
        a0.x += d0 * v.x;
        a0.y += d0 * v.y;
        a1.x += d1 * v.x;
        a1.y += d1 * v.y;
    }
    cx<T> *o = a.tmp + (((int64_t)c * 2 + comp) * nth_p + I) * nph_c + j;
    o[0] = a0;
    o[1] = a1;
}

// Gc[cc][i][j] += sum_I A/B[I][i] tmp[cc][I][j or j +- h]
template <typename T, int BS>
__global__ void __launch_bounds__(BS) k_dn_theta1(const JobList<ThetaJob<T>> jl) {
    extern __shared__ unsigned char lds_raw[];
    int local;
    const ThetaJob<T> &a = job_of(jl, local);
    const int nth_c = a.nth_c, nph_c = a.nph_c, nth_p = a.nth_p;
    T *As = reinterpret_cast<T *>(lds_raw);   // [nth_p][nth_c]
    T *Bs = As + nth_p * nth_c;
    for (int t = threadIdx.x; t < nth_p * nth_c; t += BS) {
        As[t] = a.A[t];
        Bs[t] = a.B[t];
    }
    __syncthreads();
    const int h = nph_c / 2, nc2 = (nth_c + 1) / 2;
    const int id = local * BS + (int)threadIdx.x;
    if (id >= a.ncc * nc2 * h) return;
    const int j = id % h;
    const int i = 2 * ((id / h) % nc2);
    const int64_t cc = id / (h * nc2);
    const bool two = i + 1 < nth_c;
    const int i1 = two ? i + 1 : i;
    const cx<T> *g = a.in + cc * nth_p * nph_c;
    cx<T> a0 = {0, 0}, a1 = {0, 0}, b0 = {0, 0}, b1 = {0, 0};   // rows i, i1; azimuths j, j + h
    for (int I = 0; I < nth_p; ++I) {
        const T p0 = As[I * nth_c + i], q0 = Bs[I * nth_c + i];
        const T p1 = As[I * nth_c + i1], q1 = Bs[I * nth_c + i1];
        const cx<T> g1 = g[I * nph_c + j], g2 = g[I * nph_c + j + h];
        a0.x += p0 * g1.x + q0 * g2.x;
        a0.y += p0 * g1.y + q0 * g2.y;
        b0.x += q0 * g1.x + p0 * g2.x;
        b0.y += q0 * g1.y + p0 * g2.y;
        a1.x += p1 * g1.x + q1 * g2.x;
        a1.y += p1 * g1.y + q1 * g2.y;
        b1.x += q1 * g1.x + p1 * g2.x;
        b1.y += q1 * g1.y + p1 * g2.y;
    }
    cx<T> *o = a.out + (cc * nth_c + i) * nph_c;
    cx<T> v = o[j];
    o[j] = {v.x + a0.x, v.y + a0.y};
    v = o[j + h];
    o[j + h] = {v.x + b0.x, v.y + b0.y};
    if (two) {
        v = o[nph_c + j];
        o[nph_c + j] = {v.x + a1.x, v.y + a1.y};
        v = o[nph_c + j + h];
        o[nph_c + j + h] = {v.x + b1.x, v.y + b1.y};
    }
}

// ---------------------------------------------------------------------------
// One right-hand side, a whole downward level transition per kernel: the phi
// and theta stages fused, their intermediate kept in LDS (no round trip
// through memory).  Both stages are independent across the azimuth pairs
// (j, j + h) of the child, so a (child, component) is split into chunks of
// azimuth pairs with no work repeated between chunks; the host picks the
// chunk count so that a coarse level still yields enough workgroups to fill
// the chip.  (Fusing the upward transition the same way measured slower than
// its two separate stages: its phi stage sums over the eight children.)
template <typename T>
struct FusedDnJob {   // Gc[c][comp][i][j] += (A, B)^T D^T (shift_dn Gp)
    int nchild, nth_c, nph_c, nth_p, nph_p, cols;    // cols: azimuth pairs per workgroup
    const T *A, *B, *D;
    const int *parent, *child_slot;
    const cx<T> *shift, *Gp;
    cx<T> *Gc;
};

// LDS bytes of one fused workgroup (the host checks them against the limit)
template <typename T>
__host__ __device__ inline size_t fused_dn_lds(int nth_c, int nth_p, int nph_p, int cols) {
    const size_t nt = ((size_t)nph_p * 2 * cols + 2 * (size_t)nth_p * nth_c + 1) & ~(size_t)1;
    return nt * sizeof(T) + ((size_t)nth_p * nph_p + (size_t)nth_p * 2 * cols) * 2 * sizeof(T);
}

template <typename T>
__global__ void __launch_bounds__(WG) k_dn_fused1(const JobList<FusedDnJob<T>> jl) {
    extern __shared__ unsigned char lds_raw[];
    int local;
    const FusedDnJob<T> &a = job_of(jl, local);
    const int nth_c = a.nth_c, nph_c = a.nph_c, nth_p = a.nth_p, nph_p = a.nph_p, cols = a.cols;
    const int h = nph_c / 2;
    const int nchunk = (h + cols - 1) / cols;
    const int chunk = local % nchunk, cc = local / nchunk;   // cc = child * 2 + component
    const int c = cc >> 1;
    const int j0 = chunk * cols, nj = h - j0 < cols ? h - j0 : cols;
    const int Kc = nth_c * nph_c, Kp = nth_p * nph_p, nj2 = 2 * nj;
    T *Ds = reinterpret_cast<T *>(lds_raw);   // [nph_p][2 nj]: columns j0.. and j0 + h.. of D
    T *As = Ds + nph_p * 2 * cols;            // [nth_p][nth_c]
    T *Bs = As + nth_p * nth_c;
    cx<T> *gs = reinterpret_cast<cx<T> *>(Ds + ((nph_p * 2 * cols + 2 * nth_p * nth_c + 1) & ~1));   // [nth_p][nph_p]
    cx<T> *ts = gs + Kp;                                                                              // [nth_p][2 nj]
    for (int t = threadIdx.x; t < nph_p * nj2; t += WG) {
        const int J = t / nj2, jj = t - J * nj2;
        Ds[t] = a.D[J * nph_c + (jj < nj ? j0 + jj : j0 + h + jj - nj)];
    }
    for (int t = threadIdx.x; t < nth_p * nth_c; t += WG) {
        As[t] = a.A[t];
        Bs[t] = a.B[t];
    }
    const cx<T> *g = a.Gp + ((int64_t)a.parent[c] * 2 + (cc & 1)) * Kp;
    const cx<T> *sh = a.shift + (size_t)a.child_slot[c] * Kp;
    for (int t = threadIdx.x; t < Kp; t += WG) gs[t] = cmul(sh[t], g[t]);
    __syncthreads();
    for (int t = threadIdx.x; t < nth_p * nj2; t += WG) {
        const int I = t / nj2, jj = t - I * nj2;
        const cx<T> *grow = gs + I * nph_p;
        cx<T> v = {0, 0};
        for (int J = 0; J < nph_p; ++J) {
            const T d = Ds[J * nj2 + jj];
            const cx<T> x = grow[J];
            v.x = fmad(d, x.x, v.x);
            v.y = fmad(d, x.y, v.y);
        }
        ts[t] = v;
    }
    __syncthreads();
    cx<T> *o = a.Gc + (int64_t)cc * Kc;
    for (int t = threadIdx.x; t < nth_c * nj; t += WG) {
        const int i = t / nj, jl = t - i * nj;
        cx<T> u = {0, 0}, v = {0, 0};   // azimuths j0 + jl and j0 + jl + h of row i
        for (int I = 0; I < nth_p; ++I) {
            const T pa = As[I * nth_c + i], pb = Bs[I * nth_c + i];
            const cx<T> g1 = ts[I * nj2 + jl], g2 = ts[I * nj2 + nj + jl];
            u.x = fmad(pa, g1.x, fmad(pb, g2.x, u.x));
            u.y = fmad(pa, g1.y, fmad(pb, g2.y, u.y));
            v.x = fmad(pb, g1.x, fmad(pa, g2.x, v.x));
            v.y = fmad(pb, g1.y, fmad(pa, g2.y, v.y));
        }
        const int j = j0 + jl;
        cx<T> w = o[i * nph_c + j];
        o[i * nph_c + j] = {w.x + u.x, w.y + u.y};
        w = o[i * nph_c + j + h];
        o[i * nph_c + j + h] = {w.x + v.x, w.y + v.y};
    }
}

// ---------------------------------------------------------------------------
// Diagonal translation over the interaction lists: G_b = sum T(X_bb') S_b'.
// Threads are flattened over (box, direction, rhs), rhs fastest: the R
// threads of a direction share every translation-table load.
template <typename T>
__global__ void __launch_bounds__(WG) k_translate(int nbox, int K, int R, const int *__restrict__ il_ptr,
                                                  const int *__restrict__ il_src, const int *__restrict__ il_off,
                                                  const cx<T> *__restrict__ trans, const cx<T> *__restrict__ S,
                                                  cx<T> *__restrict__ G) {
    const int64_t id = (int64_t)blockIdx.x * WG + threadIdx.x;
    const int64_t KR = (int64_t)K * R;
    if (id >= (int64_t)nbox * KR) return;
    const int b = (int)(id / KR);
    const int kr = (int)(id % KR);
    const int k = kr / R;
    cx<T> gt = {0, 0}, gp = {0, 0};
    const int q1 = il_ptr[b + 1];
    int q = il_ptr[b];
    for (; q + 1 < q1; q += 2) {
        const int s0 = il_src[q], s1 = il_src[q + 1];
        const cx<T> t0 = trans[(size_t)il_off[q] * K + k], t1 = trans[(size_t)il_off[q + 1] * K + k];
        const cx<T> a0 = S[(size_t)s0 * 2 * KR + kr], b0 = S[(size_t)s0 * 2 * KR + KR + kr];
        const cx<T> a1 = S[(size_t)s1 * 2 * KR + kr], b1 = S[(size_t)s1 * 2 * KR + KR + kr];
        cfma(gt, t0, a0);
        cfma(gp, t0, b0);
        cfma(gt, t1, a1);
        cfma(gp, t1, b1);
    }
    if (q < q1) {
        const int s0 = il_src[q];
        const cx<T> t0 = trans[(size_t)il_off[q] * K + k];
        cfma(gt, t0, S[(size_t)s0 * 2 * KR + kr]);
        cfma(gp, t0, S[(size_t)s0 * 2 * KR + KR + kr]);
    }
    G[(size_t)b * 2 * KR + kr] = gt;
    G[(size_t)b * 2 * KR + KR + kr] = gp;
}

// Translation for one right-hand side, every level of every region in one
// launch (the entries of TransLevels are (region, level) pairs).
// A workgroup takes one box and 64 directions; its four wavefronts split the
// box's interaction list (entries q = w, w + 4, ...: the source and offset ids
// are wave-uniform scalar loads) and are summed through LDS.  Workgroups are
// numbered so that each of the 8 XCDs (which take workgroups round-robin)
// receives a contiguous range of boxes in Morton order, whose source patterns
// then stay in that XCD's L2.
constexpr int TRANS_MAXJOB = 16;   // (region, level) entries of one launch
template <typename T>
struct TransLevels {
    int nlev, nblk;
    int blk0[TRANS_MAXJOB + 1];   // first workgroup of each level
    int K[TRANS_MAXJOB], nkc[TRANS_MAXJOB];
    const int *il_ptr[TRANS_MAXJOB], *il_src[TRANS_MAXJOB], *il_off[TRANS_MAXJOB];
    const cx<T> *trans[TRANS_MAXJOB], *S[TRANS_MAXJOB];
    cx<T> *G[TRANS_MAXJOB];
};

template <typename T>
__global__ void __launch_bounds__(WG) k_translate1(const TransLevels<T> tl) {
    __shared__ cx<T> part[WAVES][2][64];
    const int per = (tl.nblk + 7) / 8;
    const int id = (blockIdx.x % 8) * per + blockIdx.x / 8;
    if (id >= tl.nblk) return;   // whole workgroup: no barrier is reached
    int L = 0;
    while (L + 1 < tl.nlev && id >= tl.blk0[L + 1]) ++L;
    const int local = id - tl.blk0[L];
    const int K = tl.K[L];
    const int b = local / tl.nkc[L];
    const int k = (local % tl.nkc[L]) * 64 + (threadIdx.x & 63);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int *src = tl.il_src[L], *off = tl.il_off[L];
    const cx<T> *S = tl.S[L], *tr = tl.trans[L];
    const int kk = k < K ? k : K - 1;   // lanes past K load a valid sample, their sums are dropped
    cx<T> gt = {0, 0}, gp = {0, 0}, ht = {0, 0}, hp = {0, 0};
    const int q1 = tl.il_ptr[L][b + 1];
    int q = tl.il_ptr[L][b] + w;
    for (; q + WAVES < q1; q += 2 * WAVES) {
        const int s0 = __builtin_amdgcn_readfirstlane(src[q]), s1 = __builtin_amdgcn_readfirstlane(src[q + WAVES]);
        const int o0 = __builtin_amdgcn_readfirstlane(off[q]), o1 = __builtin_amdgcn_readfirstlane(off[q + WAVES]);
        const cx<T> t0 = tr[(size_t)o0 * K + kk], t1 = tr[(size_t)o1 * K + kk];
        const cx<T> a0 = S[(size_t)s0 * 2 * K + kk], b0 = S[(size_t)s0 * 2 * K + K + kk];
        const cx<T> a1 = S[(size_t)s1 * 2 * K + kk], b1 = S[(size_t)s1 * 2 * K + K + kk];
        cfma(gt, t0, a0);
        cfma(gp, t0, b0);
        cfma(ht, t1, a1);
        cfma(hp, t1, b1);
    }
    if (q < q1) {
        const int s0 = __builtin_amdgcn_readfirstlane(src[q]), o0 = __builtin_amdgcn_readfirstlane(off[q]);
        const cx<T> t0 = tr[(size_t)o0 * K + kk];
        cfma(gt, t0, S[(size_t)s0 * 2 * K + kk]);
        cfma(gp, t0, S[(size_t)s0 * 2 * K + K + kk]);
    }
    const int lane = threadIdx.x & 63;
    part[w][0][lane] = {gt.x + ht.x, gt.y + ht.y};
    part[w][1][lane] = {gp.x + hp.x, gp.y + hp.y};
    __syncthreads();
    if (threadIdx.x < 128) {
        const int comp = threadIdx.x >> 6;
        cx<T> v = part[0][comp][lane];
#pragma unroll
        for (int i = 1; i < WAVES; ++i) {
            v.x += part[i][comp][lane].x;
            v.y += part[i][comp][lane].y;
        }
        if (k < K) tl.G[L][(size_t)b * 2 * K + comp * K + k] = v;
    }
}

// The same for one right-hand side with the boxes grouped by parent: the
// siblings share most of their interaction lists, so a workgroup (one group,
// 64 directions) loads every candidate source sample once and applies it to
// each sibling whose list holds it.  The four wavefronts split the candidates;
// a candidate's translation samples are all requested before they are used,
// and the wavefronts' partial sums are added in LDS one wavefront at a time.
template <typename T>
struct TransGroups {
    int nlev, nblk;
    int blk0[TRANS_MAXJOB + 1];
    int K[TRANS_MAXJOB], nkc[TRANS_MAXJOB];
    const int *grp_dst[TRANS_MAXJOB], *cand_ptr[TRANS_MAXJOB], *cand_src[TRANS_MAXJOB], *cand_off[TRANS_MAXJOB];
    const cx<T> *trans[TRANS_MAXJOB], *S[TRANS_MAXJOB];
    cx<T> *G[TRANS_MAXJOB];
};

// One workgroup of the grouped single-RHS translation; `blk` is its index in
// the launch's own numbering (XCD-contiguous renumbering applied here), `red`
// an LDS buffer of 8 x 2 x 64 complex numbers.
template <typename T>
__device__ __forceinline__ void translate_grp1_block(const TransGroups<T> &tg, int blk, cx<T> (*red)[2][64]) {
    const int per = (tg.nblk + 7) / 8;
    const int id = (blk % 8) * per + blk / 8;
    if (id >= tg.nblk) return;   // whole workgroup
    int L = 0;
    while (L + 1 < tg.nlev && id >= tg.blk0[L + 1]) ++L;
    const int local = id - tg.blk0[L];
    const int K = tg.K[L];
    const int g = local / tg.nkc[L];
    const int lane = threadIdx.x & 63;
    const int k0 = (local % tg.nkc[L]) * 64;
    const int kk = k0 + lane < K ? k0 + lane : K - 1;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int *cs = tg.cand_src[L], *co = tg.cand_off[L];
    const cx<T> *S = tg.S[L], *tr = tg.trans[L];
    cx<T> acc[8][2];
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[j][0] = acc[j][1] = cx<T>{0, 0};
    const int c1 = tg.cand_ptr[L][g + 1];
    for (int c = tg.cand_ptr[L][g] + w; c < c1; c += WAVES) {
        const int s = __builtin_amdgcn_readfirstlane(cs[c]);
        const cx<T> a = S[(size_t)s * 2 * K + kk], b = S[(size_t)s * 2 * K + K + kk];
        int o[8];
        cx<T> t[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            o[j] = __builtin_amdgcn_readfirstlane(co[(int64_t)c * 8 + j]);
            t[j] = o[j] >= 0 ? tr[(size_t)o[j] * K + kk] : cx<T>{0, 0};
        }
#pragma unroll
        for (int j = 0; j < 8; ++j)
            if (o[j] >= 0) {
                cfma(acc[j][0], t[j], a);
                cfma(acc[j][1], t[j], b);
            }
    }
    for (int step = 0; step < WAVES; ++step) {
        if (w == step) {
#pragma unroll
            for (int j = 0; j < 8; ++j)
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    cx<T> v = acc[j][q];
                    if (step > 0) {
                        v.x += red[j][q][lane].x;
                        v.y += red[j][q][lane].y;
                    }
                    red[j][q][lane] = v;
                }
        }
        __syncthreads();
    }
    const int *dst = tg.grp_dst[L] + (int64_t)g * 8;
    cx<T> *G = tg.G[L];
    for (int t = threadIdx.x; t < 8 * 2 * 64; t += WG) {
        const int j = t >> 7, q = (t >> 6) & 1, ln = t & 63;
        const int d = dst[j];
        if (d >= 0 && k0 + ln < K) G[(size_t)d * 2 * K + q * K + k0 + ln] = red[j][q][ln];
    }
}

template <typename T>
__global__ void __launch_bounds__(WG) k_translate_grp1(const TransGroups<T> tg) {
    __shared__ cx<T> red[8][2][64];
    translate_grp1_block(tg, (int)blockIdx.x, red);
}

// Rows of the single-RHS near product as workgroups of WAVES rows: grp holds
// (box, row group) per workgroup, only groups with at least one row.
template <typename T>
struct NearRows {
    NearArgs<T> a;
    const int *grp;
    int ngrp;
};

// One right-hand side: up to three independent kinds of work in one launch,
// each too small to fill the chip alone or able to fill what another leaves
// idle: an upward phi stage (the coarsest: parents at level 2), translations
// that do not wait for it, and the near-field product, which depends on
// nothing in the far field.  Workgroups come in runs of eight (one per XCD);
// phi and translation runs alternate, and the near runs follow all of them,
// so the few workgroups of a small translation level start first and the
// near product's fill the rest of the chip.  Each kind keeps its own
// numbering; an empty kind takes no runs.  NEAR = false compiles the near
// kind out; GEN: the near rows are general blocks [[A, -B], [D, C]].
template <typename T, bool NEAR, bool GEN = false>
__global__ void __launch_bounds__(WG) k_near_up_phi1_translate1(const JobList<UpPhiJob<T>> jl,
                                                                const TransGroups<T> tg, const NearRows<T> nr) {
    extern __shared__ unsigned char lds_raw[];
    const int nphi = jl.blk0[jl.n];
    const int n8a = (nphi + 7) / 8, n8b = (tg.nblk + 7) / 8;
    const int within = blockIdx.x % 8;
    int run = blockIdx.x / 8;
    if (NEAR && run >= n8a + n8b) {
        const int g = 8 * (run - n8a - n8b) + within;
        if (g < nr.ngrp)
            near_block<T, 1, true, false, WAVES, GEN>(nr.a, nr.grp[2 * g], nr.grp[2 * g + 1], 0,
                                                      reinterpret_cast<cx<T> *>(lds_raw));
        return;
    }
    const int both = n8a < n8b ? n8a : n8b;
    bool phi;
    int k;
    if (run < 2 * both) {
        phi = (run & 1) == 0;
        k = run >> 1;
    } else {
        phi = n8a > n8b;
        k = both + (run - 2 * both);
    }
    const int blk = 8 * k + within;
    if (phi) {
        if (blk < nphi) up_phi1_block<T, WG>(jl, blk, lds_raw);
    } else {
        if (blk < 8 * n8b) translate_grp1_block(tg, blk, reinterpret_cast<cx<T>(*)[2][64]>(lds_raw));
    }
}

// Translation for batched right-hand sides, grouped by parent: the (up to 8)
// boxes of one parent share most of their interaction lists, so each source
// pattern sample is loaded once per group and applied to every sibling whose
// list holds it (offset id >= 0 in cand_off[c][slot]).  Lanes: rr = lane % RP
// (right-hand side, RP = R rounded up to a power of two), the rest of the
// workgroup runs over directions; blockIdx.x = group (renumbered so that each
// XCD takes a contiguous range), blockIdx.y = direction chunk, so concurrent
// workgroups share a slab of directions in cache.
template <typename T, int RP>
__global__ void __launch_bounds__(WG) k_translate_grp(int K, int R, const int *__restrict__ grp_dst,
                                                      const int *__restrict__ cand_ptr,
                                                      const int *__restrict__ cand_src,
                                                      const int *__restrict__ cand_off,
                                                      const cx<T> *__restrict__ trans, const cx<T> *__restrict__ S,
                                                      cx<T> *__restrict__ G, int ngrp) {
    constexpr int DPW = WG / RP;   // directions per workgroup
    constexpr int DW = 64 / RP;    // directions per wavefront
    // each XCD takes a contiguous range of groups (neighbouring groups share
    // most candidates, whose samples then stay in that XCD's L2); grid.x is 8 per
    const int per = (ngrp + 7) / 8;
    const int g = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    if (g >= ngrp) return;
    const int rr = threadIdx.x % RP;
    int k = blockIdx.y * DPW + threadIdx.x / RP;
    if (RP == 64) k = __builtin_amdgcn_readfirstlane(k);
    // first direction of this wavefront (wave-uniform)
    const int kw = __builtin_amdgcn_readfirstlane((int)(blockIdx.y * DPW + (threadIdx.x >> 6) * DW));
    const int q = (threadIdx.x & 63) / RP;   // this lane's direction within the wavefront
    if (k >= K || rr >= R) return;
    const int64_t KR = (int64_t)K * R;
    const int64_t kr = (int64_t)k * R + rr;
    cx<T> acc[8][2];
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[j][0] = acc[j][1] = cx<T>{0, 0};
    const int c1 = cand_ptr[g + 1];
    int c = cand_ptr[g];
    cx<T> s0 = {0, 0}, s1 = {0, 0};
    if (c < c1) {
        const int64_t base = (int64_t)cand_src[c] * 2 * KR + kr;
        s0 = S[base];
        s1 = S[base + KR];
    }
    for (; c < c1; ++c) {
        // the next candidate's samples are in flight while this one is applied
        cx<T> n0 = {0, 0}, n1 = {0, 0};
        if (c + 1 < c1) {
            const int64_t base = (int64_t)cand_src[c + 1] * 2 * KR + kr;
            n0 = S[base];
            n1 = S[base + KR];
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int o = cand_off[(int64_t)c * 8 + j];
            if (o >= 0) {
                cx<T> t;
                if constexpr (RP >= 16 && RP < 64) {
                    // two or four directions per wavefront: uniform loads of
                    // their samples, each lane takes its own
                    const cx<T> *row = trans + (int64_t)o * K + kw;
                    t = row[0];
#pragma unroll
                    for (int d = 1; d < DW; ++d) {
                        const cx<T> td = kw + d < K ? row[d] : cx<T>{0, 0};
                        if (q == d) t = td;
                    }
                } else {
                    t = trans[(int64_t)o * K + k];
                }
                cfma(acc[j][0], t, s0);
                cfma(acc[j][1], t, s1);
            }
        }
        s0 = n0;
        s1 = n1;
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int d = grp_dst[g * 8 + j];
        if (d >= 0) {
            G[(int64_t)d * 2 * KR + kr] = acc[j][0];
            G[(int64_t)d * 2 * KR + KR + kr] = acc[j][1];
        }
    }
}

// ---------------------------------------------------------------------------
// Receive at the finest level: y_E += s sum_k R.G, y_H += (s/et) sum_k R.(k x G)
// for a tile of RT right-hand sides; one wavefront per edge, lane = rr + RT kg
// (kg: direction group), reduction over the direction groups.
// NRM (JMCFIE / CNF): with the rotated test functions' patterns N as well,
// y_J += (c s R.G + N.(k x G)) / et and y_M += c s R.(k x G) - N.G, with
// c = tang = -1 (JMCFIE) or 0 (CNF): the fields E ~ G, H ~ (k x G) / et
// tested as the N-MFIE and N-EFIE rows minus the T-EFIE / et and et T-MFIE
// rows.
template <typename T, bool NRM>
__device__ __forceinline__ void receive_add(cx<T> &ye, cx<T> &yh, T s, cx<T> aE, cx<T> aH, cx<T> nE, cx<T> nH,
                                            cx<T> inv_et, T tang) {
    if (!NRM) {
        const cx<T> hh = cmul(aH, inv_et);
        ye.x += s * aE.x;
        ye.y += s * aE.y;
        yh.x += s * hh.x;
        yh.y += s * hh.y;
    } else {
        const T ts = tang * s;
        const cx<T> jj = cmul(cx<T>{ts * aE.x + nH.x, ts * aE.y + nH.y}, inv_et);
        ye.x += jj.x;
        ye.y += jj.y;
        yh.x += ts * aH.x - nE.x;
        yh.y += ts * aH.y - nE.y;
    }
}
template <typename T, bool NRM>
__device__ __forceinline__ void receive_store(cx<T> *y, int64_t iE, int64_t iH, T s, cx<T> aE, cx<T> aH, cx<T> nE,
                                              cx<T> nH, cx<T> inv_et, T tang) {
    cx<T> ye = y[iE], yh = y[iH];
    receive_add<T, NRM>(ye, yh, s, aE, aH, nE, nH, inv_et, tang);
    y[iE] = ye;
    y[iH] = yh;
}

template <typename T, int RT, bool LOSSY, bool NRM>
__global__ void __launch_bounds__(WG) k_receive(int K, int R, const int *__restrict__ edge_ptr,
                                                const int *__restrict__ edge_pos, const int *__restrict__ edge_sign,
                                                const cx<T> *__restrict__ tx, const cx<T> *__restrict__ rx,
                                                const cx<T> *__restrict__ nx, cx<T> inv_et, T tang,
                                                const cx<T> *__restrict__ G, cx<T> *__restrict__ y) {
    constexpr int NKG = 64 / RT;
    const int b = blockIdx.x;
    const int rhs0 = blockIdx.y * RT;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int rr = lane % RT, kg = lane / RT;
    const int64_t KR = (int64_t)K * R;
    const cx<T> *g = G + (size_t)b * 2 * KR + rhs0 + rr;
    for (int ie = edge_ptr[b] + wave; ie < edge_ptr[b + 1]; ie += WAVES) {
        const cx<T> *Rp = (LOSSY ? rx : tx) + (size_t)ie * 2 * K;
        const cx<T> *Np = NRM ? nx + (size_t)ie * 2 * K : nullptr;
        cx<T> aE = {0, 0}, aH = {0, 0}, nE = {0, 0}, nH = {0, 0};
        for (int k = kg; k < K; k += NKG) {
            cx<T> rt = Rp[k], rp = Rp[K + k];
            if (!LOSSY) {
                rt = cconj(rt);
                rp = cconj(rp);
            }
            const cx<T> gt = g[(size_t)k * R], gp = g[KR + (size_t)k * R];
            cfma(aE, rt, gt);
            cfma(aE, rp, gp);
            cfms(aH, rt, gp);
            cfma(aH, rp, gt);
            if (NRM) {
                cx<T> nt = Np[k], np = Np[K + k];
                if (!LOSSY) {
                    nt = cconj(nt);
                    np = cconj(np);
                }
                cfma(nE, nt, gt);
                cfma(nE, np, gp);
                cfms(nH, nt, gp);
                cfma(nH, np, gt);
            }
        }
        aE.x = group_sum<RT>(aE.x);
        aE.y = group_sum<RT>(aE.y);
        aH.x = group_sum<RT>(aH.x);
        aH.y = group_sum<RT>(aH.y);
        if (NRM) {
            nE.x = group_sum<RT>(nE.x);
            nE.y = group_sum<RT>(nE.y);
            nH.x = group_sum<RT>(nH.x);
            nH.y = group_sum<RT>(nH.y);
        }
        if (lane < RT) {
            const int p = edge_pos[ie];
            const int64_t iE = (int64_t)(2 * p) * R + rhs0 + rr, iH = iE + R;
            receive_store<T, NRM>(y, iE, iH, (T)edge_sign[ie], aE, aH, nE, nH, inv_et, tang);
        }
    }
}

// Receive at the finest level for one right-hand side.  The region's edge
// list (edges grouped by box) is cut into groups of eight consecutive edges,
// one group per wavefront, so every wavefront has the same work whatever the
// box sizes: eight lanes per edge, each lane two adjacent directions per step
// (one 16-byte load per pattern component for FP32), the incoming pattern of
// the edge's box read through the cache, and the eight partial sums of an edge
// combined by three shuffles.  K is even (K = 2 (L + 1)^2), so the pairs
// never straddle the theta/phi halves.
template <typename T>
struct Rcv1Region {
    int ne, K, nwaves;                   // region edge list entries, directions, ceil(ne / 8)
    const int *edge_box, *edge_pos, *edge_sign;
    const cx<T> *tab, *nx;               // receive table; rotated-test table (NRM)
    int conj;                            // 1: the tables are in transmit form (real k)
    cx<T> inv_et;
    const cx<T> *G;
};

// This lane's share (directions 2 sub, 2 sub + 1, + 16 ...) of the receive
// sums of entry ie of a region's edge list.
// Gf: the region's incoming patterns at the finest level.
template <typename T, bool NRM>
__device__ __forceinline__ void receive1_sums(const Rcv1Region<T> &rg, const cx<T> *Gf, int ie, int sub, cx<T> &aE,
                                              cx<T> &aH, cx<T> &nE, cx<T> &nH) {
    const int K = rg.K;
    {
        const cx<T> *Rp = rg.tab + (size_t)ie * 2 * K;
        const cx<T> *Np = NRM ? rg.nx + (size_t)ie * 2 * K : nullptr;
        const cx<T> *g = Gf + (size_t)rg.edge_box[ie] * 2 * K;
        const bool cj = rg.conj != 0;
#pragma unroll 3
        for (int k = 2 * sub; k < K; k += 16) {
            cx<T> rt0 = Rp[k], rt1 = Rp[k + 1], rp0 = Rp[K + k], rp1 = Rp[K + k + 1];
            if (cj) {
                rt0 = cconj(rt0);
                rt1 = cconj(rt1);
                rp0 = cconj(rp0);
                rp1 = cconj(rp1);
            }
            const cx<T> gt0 = g[k], gt1 = g[k + 1], gp0 = g[K + k], gp1 = g[K + k + 1];
            cfma(aE, rt0, gt0);
            cfma(aE, rp0, gp0);
            cfms(aH, rt0, gp0);
            cfma(aH, rp0, gt0);
            cfma(aE, rt1, gt1);
            cfma(aE, rp1, gp1);
            cfms(aH, rt1, gp1);
            cfma(aH, rp1, gt1);
            if (NRM) {
                cx<T> nt0 = Np[k], nt1 = Np[k + 1], np0 = Np[K + k], np1 = Np[K + k + 1];
                if (cj) {
                    nt0 = cconj(nt0);
                    nt1 = cconj(nt1);
                    np0 = cconj(np0);
                    np1 = cconj(np1);
                }
                cfma(nE, nt0, gt0);
                cfma(nE, np0, gp0);
                cfms(nH, nt0, gp0);
                cfma(nH, np0, gt0);
                cfma(nE, nt1, gt1);
                cfma(nE, np1, gp1);
                cfms(nH, nt1, gp1);
                cfma(nH, np1, gt1);
            }
        }
    }
}

// the eight lanes' partial sums of an entry combined by three shuffles
template <typename T, bool NRM>
__device__ __forceinline__ void receive1_reduce(cx<T> &aE, cx<T> &aH, cx<T> &nE, cx<T> &nH) {
#pragma unroll
    for (int m = 1; m < 8; m <<= 1) {
        aE.x += __shfl_xor(aE.x, m, 64);
        aE.y += __shfl_xor(aE.y, m, 64);
        aH.x += __shfl_xor(aH.x, m, 64);
        aH.y += __shfl_xor(aH.y, m, 64);
        if (NRM) {
            nE.x += __shfl_xor(nE.x, m, 64);
            nE.y += __shfl_xor(nE.y, m, 64);
            nH.x += __shfl_xor(nH.x, m, 64);
            nH.y += __shfl_xor(nH.y, m, 64);
        }
    }
}

// One region per launch (regions that add into the same entries of y run as
// ordered launches; k_receive1_all takes all of them in one).
template <typename T, bool NRM>
__global__ void __launch_bounds__(WG) k_receive1(const Rcv1Region<T> rg, T tang, cx<T> *__restrict__ y) {
    const int lane = threadIdx.x & 63;
    const int sub = lane & 7;
    const int w = blockIdx.x * WAVES + (threadIdx.x >> 6);
    if (w >= rg.nwaves) return;          // uniform over the wavefront
    const int ie = w * 8 + (lane >> 3);
    cx<T> aE = {0, 0}, aH = {0, 0}, nE = {0, 0}, nH = {0, 0};
    if (ie < rg.ne) receive1_sums<T, NRM>(rg, rg.G, ie, sub, aE, aH, nE, nH);
    receive1_reduce<T, NRM>(aE, aH, nE, nH);
    if (ie < rg.ne && sub == 0) {
        const int p = rg.edge_pos[ie];
        receive_store<T, NRM>(y, 2 * p, 2 * p + 1, (T)rg.edge_sign[ie], aE, aH, nE, nH, rg.inv_et, tang);
    }
}

// Receive of every region in one launch (one RHS).  Eight lanes per internal
// position p, as above; the position's contributions (one per region whose
// edge list holds its edge, in region order) are added to y[p] in registers,
// in the same order and arithmetic as one launch per region, and y is read
// and written once.
constexpr int RCV_MAXREG = 8;          // regions the single launch takes
constexpr int RCV_REG_SHIFT = 28;      // ent = region << RCV_REG_SHIFT | entry
template <typename T>
struct Rcv1All {
    int npos, maxc;                      // positions; most contributions of one position
    const int *ptr, *ent;                // [npos + 1] CSR of contributions; region and entry
    const Rcv1Region<T> *reg;            // region descriptors (device memory; their G is unset)
    const cx<T> *G[RCV_MAXREG];          // incoming finest-level patterns of each region (per batch
                                         // buffers, so set at every launch)
};

template <typename T, bool NRM>
__global__ void __launch_bounds__(WG) k_receive1_all(const Rcv1All<T> ra, T tang, cx<T> *__restrict__ y) {
    const int lane = threadIdx.x & 63;
    const int sub = lane & 7;
    const int w = blockIdx.x * WAVES + (threadIdx.x >> 6);
    if (w * 8 >= ra.npos) return;        // uniform over the wavefront
    const int p = w * 8 + (lane >> 3);
    const bool live = p < ra.npos;
    const int q0 = live ? ra.ptr[p] : 0, nq = live ? ra.ptr[p + 1] - q0 : 0;
    cx<T> ye = {0, 0}, yh = {0, 0};
    if (live) {
        ye = y[2 * (int64_t)p];
        yh = y[2 * (int64_t)p + 1];
    }
    for (int c = 0; c < ra.maxc; ++c) {  // uniform trip count: the shuffles see every lane
        cx<T> aE = {0, 0}, aH = {0, 0}, nE = {0, 0}, nH = {0, 0};
        const int e = c < nq ? ra.ent[q0 + c] : 0;
        const int r = e >> RCV_REG_SHIFT, ie = e & ((1 << RCV_REG_SHIFT) - 1);
        const cx<T> *Gr = ra.G[0];
#pragma unroll
        for (int i = 1; i < RCV_MAXREG; ++i)
            if (r == i) Gr = ra.G[i];
        if (c < nq) receive1_sums<T, NRM>(ra.reg[r], Gr, ie, sub, aE, aH, nE, nH);
        receive1_reduce<T, NRM>(aE, aH, nE, nH);
        if (c < nq)
            receive_add<T, NRM>(ye, yh, (T)ra.reg[r].edge_sign[ie], aE, aH, nE, nH, ra.reg[r].inv_et, tang);
    }
    if (live && sub == 0) {
        y[2 * (int64_t)p] = ye;
        y[2 * (int64_t)p + 1] = yh;
    }
}

// ---------------------------------------------------------------------------
// Plane-wave excitation and far field on the device (FP64).  Every edge e has
// 14 quadrature points (7 on T+, 7 on T-) with position r and weighted basis
// value w f(r) stored structure-of-arrays: qr[(q * 3 + c) * ne + e].  s0[e] is
// the edge's sign with respect to region 0 (0: interior interface).

// b[r][e] = -s0 <f_e, E_inc> / eta0, b[r][ne + e] = -s0 <f_e, H_inc> eta0 / eta0
// for the wave arriving from angles[r] = (theta, phi), polarisation pol[r].
// With qn (JMCFIE / CNF: weighted n x f samples of the unsigned halves on the
// region-0 triangles), the tangential part is weighted by tang (-1 or 0) and
// the normal parts -<n x f, H_inc> (J-rows) and +<n x f, E_inc> / eta0
// (M-rows) are added.
__global__ void k_planewave_rhs(int ne, int R, const int *__restrict__ s0, const double *__restrict__ qr,
                                const double *__restrict__ qf, const double *__restrict__ qn, double tang, double k0,
                                double inv_eta0, const double *__restrict__ angles, const double *__restrict__ pol,
                                double2 *__restrict__ b) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (int64_t)ne * R) return;
    const int e = (int)(id % ne), r = (int)(id / ne);
    double2 bE = make_double2(0, 0), bH = make_double2(0, 0), nE = make_double2(0, 0), nH = make_double2(0, 0);
    const int sg = s0[e];
    if (sg != 0) {
        double st, ct, sp, cp;
        sincos(angles[2 * r], &st, &ct);
        sincos(angles[2 * r + 1], &sp, &cp);
        const double kh[3] = {-st * cp, -st * sp, -ct};
        const double pv = pol ? pol[r] : 1.0;
        const double ev[3] = {pv * ct * cp - (1.0 - pv) * sp, pv * ct * sp + (1.0 - pv) * cp, -pv * st};
        const double hv[3] = {kh[1] * ev[2] - kh[2] * ev[1], kh[2] * ev[0] - kh[0] * ev[2],
                              kh[0] * ev[1] - kh[1] * ev[0]};
        for (int q = 0; q < 14; ++q) {
            const double x = qr[(q * 3 + 0) * (int64_t)ne + e], y = qr[(q * 3 + 1) * (int64_t)ne + e],
                         z = qr[(q * 3 + 2) * (int64_t)ne + e];
            const double fx = qf[(q * 3 + 0) * (int64_t)ne + e], fy = qf[(q * 3 + 1) * (int64_t)ne + e],
                         fz = qf[(q * 3 + 2) * (int64_t)ne + e];
            double sn, cs;
            sincos(-k0 * (kh[0] * x + kh[1] * y + kh[2] * z), &sn, &cs);
            const double fe = fx * ev[0] + fy * ev[1] + fz * ev[2];
            const double fh = fx * hv[0] + fy * hv[1] + fz * hv[2];
            bE.x += fe * cs;
            bE.y += fe * sn;
            bH.x += fh * cs;
            bH.y += fh * sn;
            if (qn) {
                const double tx = qn[(q * 3 + 0) * (int64_t)ne + e], ty = qn[(q * 3 + 1) * (int64_t)ne + e],
                             tz = qn[(q * 3 + 2) * (int64_t)ne + e];
                const double te = tx * ev[0] + ty * ev[1] + tz * ev[2];
                const double th = tx * hv[0] + ty * hv[1] + tz * hv[2];
                nE.x += te * cs;
                nE.y += te * sn;
                nH.x += th * cs;
                nH.y += th * sn;
            }
        }
    }
    const double c = -(double)sg * inv_eta0 * (qn ? tang : 1.0);
    b[(int64_t)r * 2 * ne + e] = make_double2(c * bE.x - inv_eta0 * nH.x, c * bE.y - inv_eta0 * nH.y);
    b[(int64_t)r * 2 * ne + ne + e] = make_double2(c * bH.x + inv_eta0 * nE.x, c * bH.y + inv_eta0 * nE.y);
}

// Bistatic RCS: for direction d (theta, phi) and the FP64 currents x[r]
// (boundary layout), F = (-j k0 eta0 / 4 pi) [(I - rr) J^ - r x M~^] with
// J^ = sum_e s0 J_e Int f_e exp(+j k0 r.r'); sigma = 4 pi (|F_theta|^2,
// |F_phi|^2), or with FIELD the field itself: out[(rhs, dir)][4] = Re/Im
// F_theta, Re/Im F_phi.  Grid: (directions, tiles of RCS_RT right-hand sides).
constexpr int RCS_RT = 4;
template <bool FIELD>
__global__ void __launch_bounds__(256) k_far_field(int ne, int R, const int *__restrict__ s0,
                                                   const double *__restrict__ qr, const double *__restrict__ qf,
                                                   double k0, double eta0, const double *__restrict__ dirs,
                                                   const double2 *__restrict__ x, double *__restrict__ sigma,
                                                   int n_dirs) {
    __shared__ double red[4][RCS_RT * 8];
    const int d = blockIdx.x, r0 = blockIdx.y * RCS_RT;
    double st, ct, sp, cp;
    sincos(dirs[2 * d], &st, &ct);
    sincos(dirs[2 * d + 1], &sp, &cp);
    const double rh[3] = {st * cp, st * sp, ct}, th[3] = {ct * cp, ct * sp, -st}, ph[3] = {-sp, cp, 0.0};
    double acc[RCS_RT][8];   // Jt, Jp, Mt, Mp (re, im)
#pragma unroll
    for (int t = 0; t < RCS_RT; ++t)
#pragma unroll
        for (int u = 0; u < 8; ++u) acc[t][u] = 0.0;
    for (int e = threadIdx.x; e < ne; e += blockDim.x) {
        const int sg = s0[e];
        if (sg == 0) continue;
        double ftr = 0, fti = 0, fpr = 0, fpi = 0;
        for (int q = 0; q < 14; ++q) {
            const double px = qr[(q * 3 + 0) * (int64_t)ne + e], py = qr[(q * 3 + 1) * (int64_t)ne + e],
                         pz = qr[(q * 3 + 2) * (int64_t)ne + e];
            const double fx = qf[(q * 3 + 0) * (int64_t)ne + e], fy = qf[(q * 3 + 1) * (int64_t)ne + e],
                         fz = qf[(q * 3 + 2) * (int64_t)ne + e];
            double sn, cs;
            sincos(k0 * (rh[0] * px + rh[1] * py + rh[2] * pz), &sn, &cs);
            const double a = fx * th[0] + fy * th[1] + fz * th[2];
            const double b = fx * ph[0] + fy * ph[1] + fz * ph[2];
            ftr += a * cs;
            fti += a * sn;
            fpr += b * cs;
            fpi += b * sn;
        }
#pragma unroll
        for (int t = 0; t < RCS_RT; ++t) {
            if (r0 + t >= R) continue;
            const double2 J = x[(int64_t)(r0 + t) * 2 * ne + e], M = x[(int64_t)(r0 + t) * 2 * ne + ne + e];
            const double jr = sg * J.x, ji = sg * J.y, mr = sg * M.x, mi = sg * M.y;
            acc[t][0] += jr * ftr - ji * fti;
            acc[t][1] += jr * fti + ji * ftr;
            acc[t][2] += jr * fpr - ji * fpi;
            acc[t][3] += jr * fpi + ji * fpr;
            acc[t][4] += mr * ftr - mi * fti;
            acc[t][5] += mr * fti + mi * ftr;
            acc[t][6] += mr * fpr - mi * fpi;
            acc[t][7] += mr * fpi + mi * fpr;
        }
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int t = 0; t < RCS_RT; ++t)
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const double v = wave_sum(acc[t][u]);
            if (lane == 0) red[wave][t * 8 + u] = v;
        }
    __syncthreads();
    if (threadIdx.x >= RCS_RT) return;
    const int t = threadIdx.x;
    if (r0 + t >= R) return;
    double v[8];
    for (int u = 0; u < 8; ++u) v[u] = red[0][t * 8 + u] + red[1][t * 8 + u] + red[2][t * 8 + u] + red[3][t * 8 + u];
    // F_theta = pre (Jt + Mp), F_phi = pre (Jp - Mt), pre = -j k0 eta0 / 4 pi
    const double pre = k0 * eta0 / (4.0 * 3.14159265358979323846);
    const double ar = v[0] + v[6], ai = v[1] + v[7];
    const double br = v[2] - v[4], bi = v[3] - v[5];
    if (FIELD) {   // -j pre (a, b)
        double *o = sigma + ((int64_t)(r0 + t) * n_dirs + d) * 4;
        o[0] = pre * ai;
        o[1] = -pre * ar;
        o[2] = pre * bi;
        o[3] = -pre * br;
        return;
    }
    // |pre * (a)|^2 = pre^2 |a|^2 (the -j factor has unit modulus)
    const double s = 4.0 * 3.14159265358979323846 * pre * pre;
    sigma[((int64_t)(r0 + t) * n_dirs + d) * 2] = s * (ar * ar + ai * ai);
    sigma[((int64_t)(r0 + t) * n_dirs + d) * 2 + 1] = s * (br * br + bi * bi);
}

// ---------------------------------------------------------------------------
// Batched FP64 Krylov kernels.  Vector of slot s and basis index j is at
// base + j * ldj + act[s] * lds (complex FP64, N entries, internal order).

// partial[(s * nv + j) * nblk + blk] = sum over chunk of conj(V_j[s]) w[s]
__global__ void __launch_bounds__(WG) k_bdots(const double2 *__restrict__ V, int64_t ldj, int64_t lds,
                                              const double2 *__restrict__ W, const int *__restrict__ act, int N,
                                              int nv, double2 *__restrict__ partial) {
    __shared__ double2 red[WAVES];
    const int j = blockIdx.y, s = blockIdx.z;
    const double2 *v = V + (int64_t)j * ldj + (int64_t)act[s] * lds;
    const double2 *w = W + (int64_t)act[s] * lds;
    double sx = 0, sy = 0;
    for (int i = blockIdx.x * WG + threadIdx.x; i < N; i += gridDim.x * WG) {
        const double2 a = v[i], b = w[i];
        sx += a.x * b.x + a.y * b.y;
        sy += a.x * b.y - a.y * b.x;
    }
    sx = wave_sum(sx);
    sy = wave_sum(sy);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = make_double2(sx, sy);
    __syncthreads();
    if (threadIdx.x == 0) {
        double2 t = red[0];
        for (int q = 1; q < WAVES; ++q) {
            t.x += red[q].x;
            t.y += red[q].y;
        }
        partial[((int64_t)s * nv + j) * gridDim.x + blockIdx.x] = t;
    }
}

// out[i] = sum_b partial[i][b]   (one wavefront per i, fixed order)
__global__ void k_sum_partials(const double2 *__restrict__ partial, int nblk, double2 *__restrict__ out) {
    const int i = blockIdx.x, lane = threadIdx.x;
    double sx = 0, sy = 0;
    for (int b = lane; b < nblk; b += 64) {
        sx += partial[(int64_t)i * nblk + b].x;
        sy += partial[(int64_t)i * nblk + b].y;
    }
    sx = wave_sum(sx);
    sy = wave_sum(sy);
    if (lane == 0) out[i] = make_double2(sx, sy);
}

// w[s] -= sum_j V_j[s] h[s][j]
__global__ void k_bsub(const double2 *__restrict__ V, int64_t ldj, int64_t lds, int nv, const int *__restrict__ act,
                       int N, const double2 *__restrict__ h, double2 *__restrict__ W) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x, s = blockIdx.y;
    if (i >= N) return;
    double2 *w = W + (int64_t)act[s] * lds;
    double2 acc = w[i];
    for (int j = 0; j < nv; ++j) {
        const double2 v = V[(int64_t)j * ldj + (int64_t)act[s] * lds + i], c = h[(int64_t)s * nv + j];
        acc.x -= v.x * c.x - v.y * c.y;
        acc.y -= v.x * c.y + v.y * c.x;
    }
    w[i] = acc;
}

// x[s] += sum_{j < cnt[s]} Z_j[s] y[s][j]   (y has stride nv per slot)
__global__ void k_bupdate(const double2 *__restrict__ Z, int64_t ldj, int64_t lds, int nv, const int *__restrict__ cnt,
                          const int *__restrict__ act, int N, const double2 *__restrict__ y, double2 *__restrict__ X) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x, s = blockIdx.y;
    if (i >= N) return;
    double2 *x = X + (int64_t)act[s] * lds;
    double2 acc = x[i];
    for (int j = 0; j < cnt[s]; ++j) {
        const double2 v = Z[(int64_t)j * ldj + (int64_t)act[s] * lds + i], c = y[(int64_t)s * nv + j];
        acc.x += v.x * c.x - v.y * c.y;
        acc.y += v.x * c.y + v.y * c.x;
    }
    x[i] = acc;
}

// partial[s][blk] = sum |w[s]|^2
__global__ void __launch_bounds__(WG) k_bnorm2(const double2 *__restrict__ W, int64_t lds, const int *__restrict__ act,
                                               int N, double *__restrict__ partial) {
    __shared__ double red[WAVES];
    const int s = blockIdx.y;
    const double2 *w = W + (int64_t)act[s] * lds;
    double acc = 0;
    for (int i = blockIdx.x * WG + threadIdx.x; i < N; i += gridDim.x * WG) acc += w[i].x * w[i].x + w[i].y * w[i].y;
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0;
        for (int q = 0; q < WAVES; ++q) t += red[q];
        partial[(int64_t)s * gridDim.x + blockIdx.x] = t;
    }
}

__global__ void k_sum_real(const double *__restrict__ partial, int nblk, double *__restrict__ out) {
    const int i = blockIdx.x, lane = threadIdx.x;
    double acc = 0;
    for (int b = lane; b < nblk; b += 64) acc += partial[(int64_t)i * nblk + b];
    acc = wave_sum(acc);
    if (lane == 0) out[i] = acc;
}

// w[s] *= a[s]
__global__ void k_bscale(const double *__restrict__ a, const int *__restrict__ act, int64_t lds, int N,
                         double2 *__restrict__ W) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x, s = blockIdx.y;
    if (i >= N) return;
    double2 *w = W + (int64_t)act[s] * lds;
    w[i] = make_double2(a[s] * w[i].x, a[s] * w[i].y);
}

// out[s] = c[s][0] x[s] + c[s][1] y[s] + c[s][2] z[s] (z may be null; any of
// x, y, z may be out itself: every element is read before it is written)
__global__ void k_blin3(const double2 *__restrict__ c, const int *__restrict__ act, int64_t lds, int N,
                        const double2 *x, const double2 *y, const double2 *z, double2 *out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x, s = blockIdx.y;
    if (i >= N) return;
    const int64_t o = (int64_t)act[s] * lds + i;
    const double2 c0 = c[3 * s], c1 = c[3 * s + 1], c2 = c[3 * s + 2];
    const double2 a = x[o], b = y[o];
    double2 r = make_double2(c0.x * a.x - c0.y * a.y + c1.x * b.x - c1.y * b.y,
                             c0.x * a.y + c0.y * a.x + c1.x * b.y + c1.y * b.x);
    if (z) {
        const double2 d = z[o];
        r.x += c2.x * d.x - c2.y * d.y;
        r.y += c2.x * d.y + c2.y * d.x;
    }
    out[o] = r;
}

// y[s] = b[s] - y[s]
__global__ void k_brsub(const double2 *__restrict__ Bv, const int *__restrict__ act, int64_t lds, int N,
                        double2 *__restrict__ Y) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x, s = blockIdx.y;
    if (i >= N) return;
    const double2 b = Bv[(int64_t)act[s] * lds + i];
    double2 *y = Y + (int64_t)act[s] * lds;
    y[i] = make_double2(b.x - y[i].x, b.y - y[i].y);
}

// boundary FP64 [2E] <-> internal FP64 [2E] for one vector
__global__ void k_perm_in(const double2 *__restrict__ xb, const int *__restrict__ pos, int ne,
                          double2 *__restrict__ xi) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    const int p = pos[e];
    xi[2 * p] = xb[e];
    xi[2 * p + 1] = xb[ne + e];
}
__global__ void k_perm_out(const double2 *__restrict__ xi, const int *__restrict__ pos, int ne,
                           double2 *__restrict__ xb) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    const int p = pos[e];
    xb[e] = xi[2 * p];
    xb[ne + e] = xi[2 * p + 1];
}

}  // namespace sfmm
