// HIP kernels and device orchestration for gfx950 (MI355X): the MLFMM-
// accelerated PMCHWT product, the ILU(0) solves and restarted GMRES.
//
// Data layout in HBM (internal order = finest boxes in colour/Morton order,
// canonical edge order inside a box; every edge position p holds the pair
// (J_p, M~_p) as two consecutive complex numbers):
//   x, y            [2 ne] complex T
//   near matrix     per finest box, row-major [n_b][nc_b] planes A, B, C of
//                   complex T (block [[A,-B],[B,C]] per edge pair)
//   ILU(0) factors  per finest box, row-major [2 n_b][2 nc_b] complex T,
//                   folded with the inverse diagonal-block factors
//   patterns        per region, [n_edges_r][2][K_f] complex T (theta, phi)
//   level arrays    per region and level, [n_boxes][2][K_l] complex T
//   translations    per region and level, [343 offsets][K_l] complex T
// T is float (FP32 products) or double (FP64 products); Krylov vectors and
// all reductions of the solver are FP64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "device.hpp"

namespace sfmm {

#define HIPCHK(expr)                                                                             \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            throw Error(SFMM_E_DEVICE, std::string(#expr) + " failed: " + hipGetErrorString(e_)); \
    } while (0)

#define LAUNCHCHK() HIPCHK(hipGetLastError())

template <typename T>
struct alignas(2 * sizeof(T)) cx {
    T x, y;
};

template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ void cfma(cx<T> &acc, cx<T> a, cx<T> b) {
    acc.x += a.x * b.x - a.y * b.y;
    acc.y += a.x * b.y + a.y * b.x;
}
template <typename T>
__device__ __forceinline__ void cfms(cx<T> &acc, cx<T> a, cx<T> b) {  // acc -= a b
    acc.x -= a.x * b.x - a.y * b.y;
    acc.y -= a.x * b.y + a.y * b.x;
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

constexpr int WG = 256;
constexpr int WAVES = WG / 64;
constexpr int MAXLEV = 21;
constexpr size_t LDS_LIMIT = 64 * 1024;

// ---------------------------------------------------------------------------
// Layout conversions.

// boundary FP64 [J(ne); M~(ne)] -> internal T pairs
template <typename T>
__global__ void k_to_internal(const double2 *__restrict__ xb, const int *__restrict__ pos, int ne,
                              cx<T> *__restrict__ xi) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    int p = pos[e];
    double2 j = xb[e], m = xb[ne + e];
    xi[2 * p] = {(T)j.x, (T)j.y};
    xi[2 * p + 1] = {(T)m.x, (T)m.y};
}

template <typename T>
__global__ void k_to_boundary(const cx<T> *__restrict__ yi, const int *__restrict__ pos, int ne,
                              double2 *__restrict__ yb) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    int p = pos[e];
    cx<T> j = yi[2 * p], m = yi[2 * p + 1];
    yb[e] = make_double2((double)j.x, (double)j.y);
    yb[ne + e] = make_double2((double)m.x, (double)m.y);
}

template <typename A, typename B>
__global__ void k_cast(const cx<A> *__restrict__ a, cx<B> *__restrict__ b, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = {(B)a[i].x, (B)a[i].y};
}

template <typename T>
__global__ void k_zero(cx<T> *__restrict__ a, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = {0, 0};
}

// ---------------------------------------------------------------------------
// Near-field product y = Z_near x.  Workgroups of RW wavefronts cover RW rows
// of one finest box (grid = boxes x row groups); the box's input columns are
// staged in LDS, one wavefront per row, lanes across columns, two independent
// accumulator sets per lane for memory-level parallelism.
constexpr int RW = 16;              // rows (wavefronts) per workgroup
constexpr int RWG = RW * 64;

// POLY = true fuses one step of the polynomial preconditioner into the
// epilogue: with q = Z_near x,  acc += x / theta  and  y = x - q / theta.
template <typename T, bool LDS, bool POLY = false>
__global__ void __launch_bounds__(RWG) k_near(const int *__restrict__ bstart, const int *__restrict__ col_ptr,
                                              const int *__restrict__ cols, const int64_t *__restrict__ val_ptr,
                                              const cx<T> *__restrict__ A, const cx<T> *__restrict__ B,
                                              const cx<T> *__restrict__ C, const cx<T> *__restrict__ x,
                                              cx<T> *__restrict__ y, cx<T> *__restrict__ acc = nullptr,
                                              cx<T> inv_theta = {0, 0}, int write_y = 1) {
    extern __shared__ unsigned char lds_raw[];
    cx<T> *xs = reinterpret_cast<cx<T> *>(lds_raw);
    const int b = blockIdx.x;
    const int r0 = bstart[b], nrow = bstart[b + 1] - r0;
    if ((int)blockIdx.y * RW >= nrow) return;          // uniform over the workgroup
    const int c0 = col_ptr[b], ncol = col_ptr[b + 1] - c0;
    if (LDS) {
        for (int t = threadIdx.x; t < ncol; t += RWG) {
            int p = cols[c0 + t];
            xs[2 * t] = x[2 * p];
            xs[2 * t + 1] = x[2 * p + 1];
        }
        __syncthreads();
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int row = blockIdx.y * RW + wave;
    if (row >= nrow) return;
    const int64_t rb = val_ptr[b] + (int64_t)row * ncol;
    auto xin = [&](int c, cx<T> &xj, cx<T> &xm) {
        if (LDS) {
            xj = xs[2 * c];
            xm = xs[2 * c + 1];
        } else {
            int p = cols[c0 + c];
            xj = x[2 * p];
            xm = x[2 * p + 1];
        }
    };
    cx<T> aE = {0, 0}, aH = {0, 0}, bE = {0, 0}, bH = {0, 0};
    int c = lane;
    for (; c + 64 < ncol; c += 128) {
        cx<T> a0 = A[rb + c], b0 = B[rb + c], c0v = C[rb + c];
        cx<T> a1 = A[rb + c + 64], b1 = B[rb + c + 64], c1v = C[rb + c + 64];
        cx<T> xj0, xm0, xj1, xm1;
        xin(c, xj0, xm0);
        xin(c + 64, xj1, xm1);
        cfma(aE, a0, xj0);
        cfms(aE, b0, xm0);
        cfma(aH, b0, xj0);
        cfma(aH, c0v, xm0);
        cfma(bE, a1, xj1);
        cfms(bE, b1, xm1);
        cfma(bH, b1, xj1);
        cfma(bH, c1v, xm1);
    }
    if (c < ncol) {
        cx<T> a0 = A[rb + c], b0 = B[rb + c], c0v = C[rb + c];
        cx<T> xj0, xm0;
        xin(c, xj0, xm0);
        cfma(aE, a0, xj0);
        cfms(aE, b0, xm0);
        cfma(aH, b0, xj0);
        cfma(aH, c0v, xm0);
    }
    aE.x = wave_sum(aE.x + bE.x);
    aE.y = wave_sum(aE.y + bE.y);
    aH.x = wave_sum(aH.x + bH.x);
    aH.y = wave_sum(aH.y + bH.y);
    if (lane == 0) {
        const int i = 2 * (r0 + row);
        if (POLY) {
            cx<T> xe = x[i], xh = x[i + 1];
            cx<T> ae = acc[i], ah = acc[i + 1];
            cfma(ae, xe, inv_theta);
            cfma(ah, xh, inv_theta);
            acc[i] = ae;
            acc[i + 1] = ah;
            if (write_y) {
                cfms(xe, aE, inv_theta);
                cfms(xh, aH, inv_theta);
                y[i] = xe;
                y[i + 1] = xh;
            }
        } else {
            y[i] = aE;
            y[i + 1] = aH;
        }
    }
}

// ---------------------------------------------------------------------------
// ILU(0) sweep over a range of boxes (one colour, or all boxes for the
// block-Jacobi variant): out_I = W_I [own_I ; other_K ...], grid = boxes x
// row groups of RW unknown rows, one wavefront per row.
template <typename T, bool LDS>
__global__ void __launch_bounds__(RWG) k_ilu(int box0, const int *__restrict__ bstart, const int *__restrict__ col_ptr,
                                             const int *__restrict__ cols, const int64_t *__restrict__ val_ptr,
                                             const cx<T> *__restrict__ W, const cx<T> *__restrict__ own,
                                             const cx<T> *__restrict__ other, cx<T> *__restrict__ out) {
    extern __shared__ unsigned char lds_raw[];
    cx<T> *us = reinterpret_cast<cx<T> *>(lds_raw);
    const int I = box0 + blockIdx.x;
    const int r0 = bstart[I], nI = bstart[I + 1] - r0;
    if ((int)blockIdx.y * RW >= 2 * nI) return;         // uniform over the workgroup
    const int c0 = col_ptr[I], nc = col_ptr[I + 1] - c0;
    const int nu = 2 * nc;
    if (LDS) {
        for (int t = threadIdx.x; t < nc; t += RWG) {
            int p = cols[c0 + t];
            const cx<T> *src = (t < nI) ? own : other;
            us[2 * t] = src[2 * p];
            us[2 * t + 1] = src[2 * p + 1];
        }
        __syncthreads();
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int row = blockIdx.y * RW + wave;
    if (row >= 2 * nI) return;
    const int64_t rb = val_ptr[I] + (int64_t)row * nu;
    auto uin = [&](int cc) -> cx<T> {
        if (LDS) return us[cc];
        int t = cc >> 1;
        const cx<T> *src = (t < nI) ? own : other;
        return src[2 * cols[c0 + t] + (cc & 1)];
    };
    cx<T> acc = {0, 0}, acc2 = {0, 0};
    int c = lane;
    for (; c + 64 < nu; c += 128) {
        cx<T> w0 = W[rb + c], w1 = W[rb + c + 64];
        cfma(acc, w0, uin(c));
        cfma(acc2, w1, uin(c + 64));
    }
    if (c < nu) cfma(acc, W[rb + c], uin(c));
    acc.x = wave_sum(acc.x + acc2.x);
    acc.y = wave_sum(acc.y + acc2.y);
    if (lane == 0) out[2 * r0 + row] = acc;
}

// ---------------------------------------------------------------------------
// Finest-level aggregation: S_b = sum_n s_n [et F_n J_n + ...] (theta, phi).
// One workgroup per box, blockDim = K rounded up to a wavefront (<= 1024,
// directions beyond it loop), the box's scaled excitations staged in LDS.
template <typename T>
__global__ void __launch_bounds__(1024) k_aggregate(int K, const int *__restrict__ edge_ptr,
                                                    const int *__restrict__ edge_pos, const int *__restrict__ edge_sign,
                                                    const cx<T> *__restrict__ tx, cx<T> et,
                                                    const cx<T> *__restrict__ x, cx<T> *__restrict__ S) {
    __shared__ cx<T> js[128], ms[128];
    const int b = blockIdx.x;
    const int e0 = edge_ptr[b], e1 = edge_ptr[b + 1];
    for (int k0 = 0; k0 < K; k0 += blockDim.x) {
        const int k = k0 + threadIdx.x;
        cx<T> st = {0, 0}, sp = {0, 0}, st2 = {0, 0}, sp2 = {0, 0};
        for (int c0 = e0; c0 < e1; c0 += 128) {
            const int cnt = min(128, e1 - c0);
            __syncthreads();
            for (int t = threadIdx.x; t < cnt; t += blockDim.x) {
                int p = edge_pos[c0 + t];
                T s = (T)edge_sign[c0 + t];
                cx<T> xj = x[2 * p], xm = x[2 * p + 1];
                cx<T> j = cmul(et, xj);
                js[t] = {s * j.x, s * j.y};
                ms[t] = {s * xm.x, s * xm.y};
            }
            __syncthreads();
            if (k < K) {
                const cx<T> *F = tx + (size_t)c0 * 2 * K + k;
                int t = 0;
                for (; t + 1 < cnt; t += 2) {
                    const cx<T> ft = F[(size_t)t * 2 * K], fp = F[(size_t)t * 2 * K + K];
                    const cx<T> gt = F[(size_t)(t + 1) * 2 * K], gp = F[(size_t)(t + 1) * 2 * K + K];
                    cfma(st, ft, js[t]);
                    cfma(st, fp, ms[t]);
                    cfma(sp, fp, js[t]);
                    cfms(sp, ft, ms[t]);
                    cfma(st2, gt, js[t + 1]);
                    cfma(st2, gp, ms[t + 1]);
                    cfma(sp2, gp, js[t + 1]);
                    cfms(sp2, gt, ms[t + 1]);
                }
                if (t < cnt) {
                    const cx<T> ft = F[(size_t)t * 2 * K], fp = F[(size_t)t * 2 * K + K];
                    cfma(st, ft, js[t]);
                    cfma(st, fp, ms[t]);
                    cfma(sp, fp, js[t]);
                    cfms(sp, ft, ms[t]);
                }
            }
        }
        if (k < K) {
            S[(size_t)b * 2 * K + k] = {st.x + st2.x, st.y + st2.y};
            S[(size_t)b * 2 * K + K + k] = {sp.x + sp2.x, sp.y + sp2.y};
        }
    }
}

// ---------------------------------------------------------------------------
// Upward pass, theta stage: for every child box, comp, parent theta row I and
// child phi column j: tmp = A f(:, j) + B f(:, j +- nph/2)  (even/odd pairing)
template <typename T>
__global__ void k_up_theta(int nchild, int nth_c, int nph_c, int nth_p, const T *__restrict__ A,
                           const T *__restrict__ B, const cx<T> *__restrict__ S, cx<T> *__restrict__ tmp) {
    const int64_t total = (int64_t)nchild * 2 * nth_p * nph_c;
    int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= total) return;
    int j = id % nph_c;
    int64_t r = id / nph_c;
    int I = r % nth_p;
    int64_t cc = r / nth_p;  // child * 2 + comp
    const int h = nph_c / 2;
    const int j1 = j < h ? j : j - h;   // lower column of the pair
    const int j2 = j1 + h;
    const T *Pa = (j < h) ? A : B;      // coefficient of column j1
    const T *Pb = (j < h) ? B : A;      // coefficient of column j2
    const cx<T> *f = S + cc * nth_c * nph_c;
    cx<T> acc = {0, 0};
    for (int i = 0; i < nth_c; ++i) {
        T a = Pa[I * nth_c + i], b = Pb[I * nth_c + i];
        cx<T> f1 = f[i * nph_c + j1], f2 = f[i * nph_c + j2];
        acc.x += a * f1.x + b * f2.x;
        acc.y += a * f1.y + b * f2.y;
    }
    tmp[id] = acc;
}

// Upward pass, phi stage + shift + sum over the children of every parent.
template <typename T>
__global__ void k_up_phi(int nparent, int nth_p, int nph_p, int nph_c, const T *__restrict__ D,
                         const int *__restrict__ child_ptr, const int *__restrict__ child_idx,
                         const int *__restrict__ child_slot, const cx<T> *__restrict__ shift,
                         const cx<T> *__restrict__ tmp, cx<T> *__restrict__ Sp) {
    const int Kp = nth_p * nph_p;
    const int64_t total = (int64_t)nparent * 2 * Kp;
    int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= total) return;
    int kk = id % Kp;
    int64_t r = id / Kp;
    int comp = r % 2;
    int P = r / 2;
    int I = kk / nph_p, J = kk % nph_p;
    cx<T> out = {0, 0};
    for (int q = child_ptr[P]; q < child_ptr[P + 1]; ++q) {
        int c = child_idx[q];
        const cx<T> *g = tmp + (((int64_t)c * 2 + comp) * nth_p + I) * nph_c;
        cx<T> v = {0, 0};
        for (int j = 0; j < nph_c; ++j) {
            T d = D[J * nph_c + j];
            v.x += d * g[j].x;
            v.y += d * g[j].y;
        }
        cfma(out, shift[child_slot[c] * Kp + kk], v);
    }
    Sp[id] = out;
}

// Downward pass, phi stage (transpose of k_up_phi): for every child box,
// tmp[c][comp][I][j] = sum_J D[J][j] shift_dn[slot][I,J] G_parent[comp][I][J]
template <typename T>
__global__ void k_dn_phi(int nchild, int nth_p, int nph_p, int nph_c, const T *__restrict__ D,
                         const int *__restrict__ parent, const int *__restrict__ child_slot,
                         const cx<T> *__restrict__ shift, const cx<T> *__restrict__ Gp,
                         cx<T> *__restrict__ tmp) {
    const int Kp = nth_p * nph_p;
    const int64_t total = (int64_t)nchild * 2 * nth_p * nph_c;
    int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= total) return;
    int j = id % nph_c;
    int64_t r = id / nph_c;
    int I = r % nth_p;
    r /= nth_p;
    int comp = r % 2;
    int c = r / 2;
    const cx<T> *g = Gp + ((int64_t)parent[c] * 2 + comp) * Kp + I * nph_p;
    const cx<T> *sh = shift + child_slot[c] * Kp + I * nph_p;
    cx<T> acc = {0, 0};
    for (int J = 0; J < nph_p; ++J) {
        cx<T> v = cmul(sh[J], g[J]);
        T d = D[J * nph_c + j];
        acc.x += d * v.x;
        acc.y += d * v.y;
    }
    tmp[id] = acc;
}

// Downward pass, theta stage (transpose of k_up_theta), accumulated into G_child.
template <typename T>
__global__ void k_dn_theta(int nchild, int nth_c, int nph_c, int nth_p, const T *__restrict__ A,
                           const T *__restrict__ B, const cx<T> *__restrict__ tmp, cx<T> *__restrict__ Gc) {
    const int64_t total = (int64_t)nchild * 2 * nth_c * nph_c;
    int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= total) return;
    int j = id % nph_c;
    int64_t r = id / nph_c;
    int i = r % nth_c;
    int64_t cc = r / nth_c;
    const int h = nph_c / 2;
    const int j1 = j < h ? j : j - h;
    const int j2 = j1 + h;
    // f(i, j1) = sum_I A[I,i] g(I, j1) + B[I,i] g(I, j2);  f(i, j2) = B g(j1) + A g(j2)
    const T *Pa = (j < h) ? A : B;
    const T *Pb = (j < h) ? B : A;
    const cx<T> *g = tmp + cc * nth_p * nph_c;
    cx<T> acc = Gc[id];
    for (int I = 0; I < nth_p; ++I) {
        T a = Pa[I * nth_c + i], b = Pb[I * nth_c + i];
        cx<T> g1 = g[I * nph_c + j1], g2 = g[I * nph_c + j2];
        acc.x += a * g1.x + b * g2.x;
        acc.y += a * g1.y + b * g2.y;
    }
    Gc[id] = acc;
}

// ---------------------------------------------------------------------------
// LDS-staged interpolation.  One workgroup per (parent box, component, chunk
// of UPR parent theta rows): for every child in turn the child pattern is
// staged in LDS, the theta stage computes only the chunk's rows into LDS, and
// the phi stage + shift accumulates the chunk's outputs in registers.
constexpr int UPR = 4;      // parent theta rows per workgroup
constexpr int UPMAX = 8;    // outputs per thread: UPR * nph_p <= WG * UPMAX

template <typename T>
__global__ void __launch_bounds__(WG) k_up_box(int nth_c, int nph_c, int nth_p, int nph_p, const T *__restrict__ A,
                                               const T *__restrict__ B, const T *__restrict__ Dt,
                                               const int *__restrict__ child_ptr, const int *__restrict__ child_idx,
                                               const int *__restrict__ child_slot, const cx<T> *__restrict__ shift,
                                               const cx<T> *__restrict__ Sc, cx<T> *__restrict__ Sp) {
    extern __shared__ unsigned char lds_raw[];
    const int Kc = nth_c * nph_c, Kp = nth_p * nph_p;
    cx<T> *fs = reinterpret_cast<cx<T> *>(lds_raw);      // [Kc]
    cx<T> *ts = fs + Kc;                                   // [UPR][nph_c]
    const int nchunk = (nth_p + UPR - 1) / UPR;
    const int P = blockIdx.x / (2 * nchunk);
    const int comp = (blockIdx.x / nchunk) % 2;
    const int I0 = (blockIdx.x % nchunk) * UPR;
    const int nI = min(UPR, nth_p - I0);
    const int nout = nI * nph_p;
    const int h = nph_c / 2;
    cx<T> acc[UPMAX];
#pragma unroll
    for (int u = 0; u < UPMAX; ++u) acc[u] = {0, 0};
    for (int q = child_ptr[P]; q < child_ptr[P + 1]; ++q) {
        const int c = child_idx[q];
        const cx<T> *f = Sc + ((size_t)c * 2 + comp) * Kc;
        __syncthreads();
        for (int t = threadIdx.x; t < Kc; t += WG) fs[t] = f[t];
        __syncthreads();
        for (int t = threadIdx.x; t < nI * nph_c; t += WG) {
            const int I = I0 + t / nph_c, j = t % nph_c;
            const int j1 = j < h ? j : j - h, j2 = j1 + h;
            const T *Pa = (j < h) ? A : B;
            const T *Pb = (j < h) ? B : A;
            cx<T> a2 = {0, 0};
            for (int i = 0; i < nth_c; ++i) {
                const T a = Pa[I * nth_c + i], b = Pb[I * nth_c + i];
                const cx<T> f1 = fs[i * nph_c + j1], f2 = fs[i * nph_c + j2];
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
                const int Il = o / nph_p, J = o % nph_p;
                const cx<T> *g = ts + Il * nph_c;
                cx<T> v = {0, 0};
                for (int j = 0; j < nph_c; ++j) {
                    const T d = Dt[(size_t)j * nph_p + J];
                    v.x += d * g[j].x;
                    v.y += d * g[j].y;
                }
                cfma(acc[u], sh[o], v);
            }
        }
    }
    cx<T> *out = Sp + ((size_t)P * 2 + comp) * Kp + I0 * nph_p;
#pragma unroll
    for (int u = 0; u < UPMAX; ++u) {
        const int o = threadIdx.x + u * WG;
        if (o < nout) out[o] = acc[u];
    }
}

// LDS-staged anterpolation: one workgroup per child box: shifted parent
// pattern -> LDS, phi transpose -> LDS, theta transpose accumulated into the
// child pattern.
template <typename T>
__global__ void __launch_bounds__(WG) k_dn_box(int nth_c, int nph_c, int nth_p, int nph_p, const T *__restrict__ A,
                                               const T *__restrict__ B, const T *__restrict__ D,
                                               const int *__restrict__ parent, const int *__restrict__ child_slot,
                                               const cx<T> *__restrict__ shift, const cx<T> *__restrict__ Gp,
                                               cx<T> *__restrict__ Gc) {
    extern __shared__ unsigned char lds_raw[];
    const int Kc = nth_c * nph_c, Kp = nth_p * nph_p;
    cx<T> *gs = reinterpret_cast<cx<T> *>(lds_raw);      // [Kp]
    cx<T> *ts = gs + Kp;                                   // [nth_p][nph_c]
    const int c = blockIdx.x;
    const int h = nph_c / 2;
    const cx<T> *sh = shift + (size_t)child_slot[c] * Kp;
    for (int comp = 0; comp < 2; ++comp) {
        const cx<T> *g = Gp + ((size_t)parent[c] * 2 + comp) * Kp;
        __syncthreads();
        for (int t = threadIdx.x; t < Kp; t += WG) gs[t] = cmul(sh[t], g[t]);
        __syncthreads();
        for (int t = threadIdx.x; t < nth_p * nph_c; t += WG) {
            const int I = t / nph_c, j = t % nph_c;
            const cx<T> *row = gs + I * nph_p;
            cx<T> acc = {0, 0};
            for (int J = 0; J < nph_p; ++J) {
                const T d = D[(size_t)J * nph_c + j];
                acc.x += d * row[J].x;
                acc.y += d * row[J].y;
            }
            ts[t] = acc;
        }
        __syncthreads();
        cx<T> *out = Gc + ((size_t)c * 2 + comp) * Kc;
        for (int t = threadIdx.x; t < Kc; t += WG) {
            const int i = t / nph_c, j = t % nph_c;
            const int j1 = j < h ? j : j - h, j2 = j1 + h;
            const T *Pa = (j < h) ? A : B;
            const T *Pb = (j < h) ? B : A;
            cx<T> acc = out[t];
            for (int I = 0; I < nth_p; ++I) {
                const T a = Pa[I * nth_c + i], b = Pb[I * nth_c + i];
                const cx<T> g1 = ts[I * nph_c + j1], g2 = ts[I * nph_c + j2];
                acc.x += a * g1.x + b * g2.x;
                acc.y += a * g1.y + b * g2.y;
            }
            out[t] = acc;
        }
    }
}

// ---------------------------------------------------------------------------
// Diagonal translation over the interaction lists: G_b = sum T(X_bb') S_b'.
// Threads are flattened over (box, direction) so no lane idles on short K.
template <typename T>
__global__ void __launch_bounds__(WG) k_translate(int nbox, int K, const int *__restrict__ il_ptr,
                                                  const int *__restrict__ il_src, const int *__restrict__ il_off,
                                                  const cx<T> *__restrict__ trans, const cx<T> *__restrict__ S,
                                                  cx<T> *__restrict__ G) {
    const int64_t id = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (id >= (int64_t)nbox * K) return;
    const int b = (int)(id / K), k = (int)(id % K);
    cx<T> gt = {0, 0}, gp = {0, 0};
    const int q1 = il_ptr[b + 1];
    int q = il_ptr[b];
    for (; q + 1 < q1; q += 2) {
        const int s0 = il_src[q], s1 = il_src[q + 1];
        const cx<T> t0 = trans[(size_t)il_off[q] * K + k], t1 = trans[(size_t)il_off[q + 1] * K + k];
        const cx<T> a0 = S[(size_t)s0 * 2 * K + k], b0 = S[(size_t)s0 * 2 * K + K + k];
        const cx<T> a1 = S[(size_t)s1 * 2 * K + k], b1 = S[(size_t)s1 * 2 * K + K + k];
        cfma(gt, t0, a0);
        cfma(gp, t0, b0);
        cfma(gt, t1, a1);
        cfma(gp, t1, b1);
    }
    if (q < q1) {
        const int s0 = il_src[q];
        const cx<T> t0 = trans[(size_t)il_off[q] * K + k];
        cfma(gt, t0, S[(size_t)s0 * 2 * K + k]);
        cfma(gp, t0, S[(size_t)s0 * 2 * K + K + k]);
    }
    G[(size_t)b * 2 * K + k] = gt;
    G[(size_t)b * 2 * K + K + k] = gp;
}

// ---------------------------------------------------------------------------
// Receive at the finest level: y_E += s sum_k R.G, y_H += (s/et) sum_k R.(k x G).
template <typename T, bool LOSSY>
__global__ void __launch_bounds__(WG) k_receive(int K, const int *__restrict__ edge_ptr,
                                                const int *__restrict__ edge_pos, const int *__restrict__ edge_sign,
                                                const cx<T> *__restrict__ tx, const cx<T> *__restrict__ rx,
                                                cx<T> inv_et, const cx<T> *__restrict__ G,
                                                cx<T> *__restrict__ y) {
    const int b = blockIdx.x;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const cx<T> *g = G + (size_t)b * 2 * K;
    for (int ie = edge_ptr[b] + wave; ie < edge_ptr[b + 1]; ie += WAVES) {
        const cx<T> *R = (LOSSY ? rx : tx) + (size_t)ie * 2 * K;
        cx<T> aE = {0, 0}, aH = {0, 0};
        for (int k = lane; k < K; k += 64) {
            cx<T> rt = R[k], rp = R[K + k];
            if (!LOSSY) {
                rt = cconj(rt);
                rp = cconj(rp);
            }
            cx<T> gt = g[k], gp = g[K + k];
            cfma(aE, rt, gt);
            cfma(aE, rp, gp);
            cfms(aH, rt, gp);
            cfma(aH, rp, gt);
        }
        aE.x = wave_sum(aE.x);
        aE.y = wave_sum(aE.y);
        aH.x = wave_sum(aH.x);
        aH.y = wave_sum(aH.y);
        if (lane == 0) {
            const int p = edge_pos[ie];
            const T s = (T)edge_sign[ie];
            cx<T> h = cmul(aH, inv_et);
            cx<T> ye = y[2 * p], yh = y[2 * p + 1];
            ye.x += s * aE.x;
            ye.y += s * aE.y;
            yh.x += s * h.x;
            yh.y += s * h.y;
            y[2 * p] = ye;
            y[2 * p + 1] = yh;
        }
    }
}

// ---------------------------------------------------------------------------
// FP64 Krylov kernels (internal order, N complex entries per vector).

// partial[j][blk] = sum_{i in chunk} conj(V_j[i]) w[i]
__global__ void __launch_bounds__(WG) k_dots(const double2 *__restrict__ V, int64_t ldv, int N,
                                             const double2 *__restrict__ w, double2 *__restrict__ partial) {
    __shared__ double2 red[WAVES];
    const int j = blockIdx.y;
    const double2 *v = V + (int64_t)j * ldv;
    double sx = 0, sy = 0;
    for (int i = blockIdx.x * WG + threadIdx.x; i < N; i += gridDim.x * WG) {
        double2 a = v[i], b = w[i];
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
        partial[(int64_t)j * gridDim.x + blockIdx.x] = t;
    }
}

// out[j] = sum_b partial[j][b]   (one wavefront per j, fixed order)
__global__ void k_sum_partials(const double2 *__restrict__ partial, int nblk, double2 *__restrict__ out) {
    const int j = blockIdx.x;
    const int lane = threadIdx.x;
    double sx = 0, sy = 0;
    for (int b = lane; b < nblk; b += 64) {
        sx += partial[(int64_t)j * nblk + b].x;
        sy += partial[(int64_t)j * nblk + b].y;
    }
    sx = wave_sum(sx);
    sy = wave_sum(sy);
    if (lane == 0) out[j] = make_double2(sx, sy);
}

// w -= sum_j V_j h[j]
__global__ void k_sub_vh(const double2 *__restrict__ V, int64_t ldv, int nv, int N, const double2 *__restrict__ h,
                         double2 *__restrict__ w) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double2 acc = w[i];
    for (int j = 0; j < nv; ++j) {
        double2 v = V[(int64_t)j * ldv + i], c = h[j];
        acc.x -= v.x * c.x - v.y * c.y;
        acc.y -= v.x * c.y + v.y * c.x;
    }
    w[i] = acc;
}

// u = sum_j V_j y[j]
__global__ void k_lincomb(const double2 *__restrict__ V, int64_t ldv, int nv, int N, const double2 *__restrict__ y,
                          double2 *__restrict__ u) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double2 acc = make_double2(0, 0);
    for (int j = 0; j < nv; ++j) {
        double2 v = V[(int64_t)j * ldv + i], c = y[j];
        acc.x += v.x * c.x - v.y * c.y;
        acc.y += v.x * c.y + v.y * c.x;
    }
    u[i] = acc;
}

// partial[blk] = sum |w|^2
__global__ void __launch_bounds__(WG) k_norm2(const double2 *__restrict__ w, int N, double *__restrict__ partial) {
    __shared__ double red[WAVES];
    double s = 0;
    for (int i = blockIdx.x * WG + threadIdx.x; i < N; i += gridDim.x * WG) {
        double2 a = w[i];
        s += a.x * a.x + a.y * a.y;
    }
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0;
        for (int q = 0; q < WAVES; ++q) t += red[q];
        partial[blockIdx.x] = t;
    }
}

__global__ void k_sum_real(const double *__restrict__ partial, int n, double *__restrict__ out) {
    const int lane = threadIdx.x;
    double s = 0;
    for (int b = lane; b < n; b += 64) s += partial[b];
    s = wave_sum(s);
    if (lane == 0) *out = s;
}

// y = a x (a real)
__global__ void k_scale(const double2 *__restrict__ x, double a, int N, double2 *__restrict__ y) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) y[i] = make_double2(a * x[i].x, a * x[i].y);
}

// y = x - y   (residual r = b - Ax with y holding Ax)
__global__ void k_rsub(const double2 *__restrict__ x, int N, double2 *__restrict__ y) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) y[i] = make_double2(x[i].x - y[i].x, x[i].y - y[i].y);
}

// y += x
__global__ void k_add(const double2 *__restrict__ x, int N, double2 *__restrict__ y) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) y[i] = make_double2(x[i].x + y[i].x, x[i].y + y[i].y);
}

// internal FP64 <-> boundary FP64 (permutation only)
__global__ void k_perm_in(const double2 *__restrict__ xb, const int *__restrict__ pos, int ne,
                          double2 *__restrict__ xi) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    int p = pos[e];
    xi[2 * p] = xb[e];
    xi[2 * p + 1] = xb[ne + e];
}
__global__ void k_perm_out(const double2 *__restrict__ xi, const int *__restrict__ pos, int ne,
                           double2 *__restrict__ xb) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    int p = pos[e];
    xb[e] = xi[2 * p];
    xb[ne + e] = xi[2 * p + 1];
}

// ---------------------------------------------------------------------------
// Host helpers

void *device_alloc(size_t bytes) {
    void *p = nullptr;
    if (bytes == 0) bytes = 16;
    hipError_t e = hipMalloc(&p, bytes);
    if (e == hipErrorOutOfMemory) throw Error(SFMM_E_OOM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    HIPCHK(e);
    return p;
}
void device_free(void *p) {
    if (p) (void)hipFree(p);
}
void copy_h2d(void *dst, const void *src, size_t bytes, void *stream) {
    HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, (hipStream_t)stream));
}
void copy_d2h(void *dst, const void *src, size_t bytes, void *stream) {
    HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, (hipStream_t)stream));
    HIPCHK(hipStreamSynchronize((hipStream_t)stream));
}
void stream_sync(void *stream) { HIPCHK(hipStreamSynchronize((hipStream_t)stream)); }

void check_device(int device) {
    int n = 0;
    HIPCHK(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) throw Error(SFMM_E_DEVICE, "no HIP device with ordinal " + std::to_string(device));
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, device));
    if (std::string(prop.gcnArchName).rfind("gfx950", 0) != 0)
        throw Error(SFMM_E_DEVICE, std::string("library built for gfx950, device is ") + prop.gcnArchName);
}

namespace {

inline unsigned nblocks(int64_t n, int bs = WG) { return (unsigned)((n + bs - 1) / bs); }

template <typename T>
cx<T> to_cx(cd v) {
    return {(T)v.real(), (T)v.imag()};
}

template <typename T>
class DeviceBodyT final : public DeviceBody {
  public:
    DeviceBodyT(const BodyHost &h, int device, void *stream) : h_(h), dev_(device), stream_((hipStream_t)stream) {
        HIPCHK(hipSetDevice(device));
        const Mesh &m = h.mesh;
        const Octree &o = h.oct;
        ne_ = m.ne;
        nb_ = o.nb;
        f_ = o.f;
        colour_ptr_ = o.colour_ptr;
        pos_ = upload(o.pos);
        bstart_ = upload(o.bstart);
        // near matrix
        near_col_ptr_ = upload(h.near.col_ptr);
        near_cols_ = upload(h.near.cols);
        near_val_ptr_ = upload(h.near.val_ptr);
        nA_ = upload_cx(h.near.A);
        nB_ = upload_cx(h.near.B);
        nC_ = upload_cx(h.near.C);
        max_ncol_ = 0;
        max_nrow_ = 0;
        precond_ = h.precond;
        for (const cd &t : h.poly) inv_theta_.push_back(to_cx<T>(1.0 / t));
        for (int b = 0; b < nb_; ++b) {
            max_ncol_ = std::max(max_ncol_, h.near.col_ptr[b + 1] - h.near.col_ptr[b]);
            max_nrow_ = std::max(max_nrow_, o.bstart[b + 1] - o.bstart[b]);
        }
        // ILU factors
        fcol_ptr_ = upload(h.ilu.fwd_col_ptr);
        fcols_ = upload(h.ilu.fwd_cols);
        fptr_ = upload(h.ilu.fwd_ptr);
        fval_ = upload_cx(h.ilu.fwd);
        bcol_ptr_ = upload(h.ilu.bwd_col_ptr);
        bcols_ = upload(h.ilu.bwd_cols);
        bptr_ = upload(h.ilu.bwd_ptr);
        bval_ = upload_cx(h.ilu.bwd);
        max_ilu_nc_ = 0;
        for (int b = 0; b < nb_ && !h.ilu.fwd_col_ptr.empty(); ++b) {
            max_ilu_nc_ = std::max(max_ilu_nc_, h.ilu.fwd_col_ptr[b + 1] - h.ilu.fwd_col_ptr[b]);
            if (!h.ilu.bwd_col_ptr.empty())
                max_ilu_nc_ = std::max(max_ilu_nc_, h.ilu.bwd_col_ptr[b + 1] - h.ilu.bwd_col_ptr[b]);
        }
        // regions
        for (size_t ri = 0; ri < o.regions.size(); ++ri) {
            const RegionTree &rt = o.regions[ri];
            const RegionTables &tb = h.tables[ri];
            Reg R;
            R.et = to_cx<T>(tb.eta);
            R.inv_et = to_cx<T>(1.0 / tb.eta);
            R.lossy = tb.lossy;
            R.nbf = (int)rt.fbox.size();
            R.edge_ptr = upload(rt.edge_ptr);
            R.edge_pos = upload(rt.edge_pos);
            R.edge_sign = upload(rt.edge_sign);
            if (f_ >= 2) {
                R.tx = upload_cx(tb.tx);
                if (tb.lossy) R.rx = upload_cx(tb.rx);
                size_t tmp_elems = 0;
                for (int l = 2; l <= f_; ++l) {
                    const Sampling &s = tb.samp[l];
                    const LevelBoxes &lv = rt.lev[l];
                    R.K[l] = s.K;
                    R.nth[l] = s.nth;
                    R.nph[l] = s.nph;
                    R.nbox[l] = (int)lv.key.size();
                    R.S[l] = alloc_cx((size_t)R.nbox[l] * 2 * s.K);
                    R.G[l] = alloc_cx((size_t)R.nbox[l] * 2 * s.K);
                    R.il_ptr[l] = upload(lv.il_ptr);
                    R.il_src[l] = upload(lv.il_src);
                    R.il_off[l] = upload(lv.il_off);
                    R.trans[l] = upload_cx(tb.trans[l]);
                    if (l >= 3) {
                        R.parent[l] = upload(lv.parent);
                        R.slot[l] = upload(lv.child_slot);
                        R.ipA[l] = upload_real(tb.ipA[l]);
                        R.ipB[l] = upload_real(tb.ipB[l]);
                        R.ipD[l] = upload_real(tb.ipD[l]);
                        {
                            const int np_p = tb.samp[l - 1].nph, np_c = s.nph;
                            std::vector<double> Dt((size_t)np_p * np_c);
                            for (int J = 0; J < np_p; ++J)
                                for (int jj = 0; jj < np_c; ++jj) Dt[(size_t)jj * np_p + J] = tb.ipD[l][(size_t)J * np_c + jj];
                            R.ipDt[l] = upload_real(Dt);
                        }
                        R.sup[l] = upload_cx(tb.shift_up[l]);
                        R.sdn[l] = upload_cx(tb.shift_dn[l]);
                        const Sampling &p = tb.samp[l - 1];
                        tmp_elems = std::max(tmp_elems, (size_t)R.nbox[l] * 2 * p.nth * s.nph);
                    }
                    if (l < f_) {
                        R.child_ptr[l] = upload(lv.child_ptr);
                        R.child_idx[l] = upload(lv.child_idx);
                    }
                }
                if (tmp_elems) R.tmp = alloc_cx(tmp_elems);
            }
            regs_.push_back(R);
        }
        const int N = 2 * ne_;
        xi_ = alloc_cx(N);
        yi_ = alloc_cx(N);
        zi_ = alloc_cx(N);
        wi_ = alloc_cx(N);
        pt_ = alloc_cx(N);
        HIPCHK(hipEventCreate(&ev0_));
        HIPCHK(hipEventCreate(&ev1_));
        for (auto &e : evs_) HIPCHK(hipEventCreate(&e));
    }

    ~DeviceBodyT() override {
        for (void *p : allocs_) device_free(p);
        if (ev0_) (void)hipEventDestroy(ev0_);
        if (ev1_) (void)hipEventDestroy(ev1_);
        for (auto &e : evs_)
            if (e) (void)hipEventDestroy(e);
    }

    void set_stream(void *s) override { stream_ = (hipStream_t)s; }
    void profile(bool enable) override {
        profiling_ = enable;
        if (enable) times_ = StageTimes();
    }
    StageTimes times() const override { return times_; }
    int64_t device_bytes() const override { return bytes_; }

    // ---- products on internal T vectors ----
    void matvec_internal(const cx<T> *x, cx<T> *y, int parts) {
        const int N = 2 * ne_;
        mark(0);
        if (parts & SFMM_PART_NEAR) {
            size_t lds = (size_t)max_ncol_ * 2 * sizeof(cx<T>);
            dim3 grid(nb_, (max_nrow_ + RW - 1) / RW);
            if (lds <= LDS_LIMIT)
                k_near<T, true><<<grid, RWG, lds, stream_>>>(bstart_, near_col_ptr_, near_cols_, near_val_ptr_, nA_, nB_, nC_, x, y);
            else
                k_near<T, false><<<grid, RWG, 0, stream_>>>(bstart_, near_col_ptr_, near_cols_, near_val_ptr_, nA_, nB_, nC_, x, y);
            LAUNCHCHK();
        } else {
            k_zero<T><<<nblocks(N), WG, 0, stream_>>>(y, N);
            LAUNCHCHK();
        }
        mark(1);
        if ((parts & SFMM_PART_FAR) && f_ >= 2) {
            for (Reg &R : regs_) {
                const int f = f_;
                const int bs = std::min(1024, ((R.K[f] + 63) / 64) * 64);
                k_aggregate<T><<<R.nbf, bs, 0, stream_>>>(R.K[f], R.edge_ptr, R.edge_pos, R.edge_sign, R.tx, R.et, x, R.S[f]);
                LAUNCHCHK();
            }
            mark(2);
            for (Reg &R : regs_) {
                for (int l = f_; l >= 3; --l) {
                    size_t lds = ((size_t)R.K[l] + (size_t)UPR * R.nph[l]) * sizeof(cx<T>);
                    if (lds <= LDS_LIMIT && UPR * R.nph[l - 1] <= WG * UPMAX) {
                        const int nchunk = (R.nth[l - 1] + UPR - 1) / UPR;
                        k_up_box<T><<<R.nbox[l - 1] * 2 * nchunk, WG, lds, stream_>>>(R.nth[l], R.nph[l], R.nth[l - 1], R.nph[l - 1],
                                                                        R.ipA[l], R.ipB[l], R.ipDt[l], R.child_ptr[l - 1],
                                                                        R.child_idx[l - 1], R.slot[l], R.sup[l], R.S[l],
                                                                        R.S[l - 1]);
                        LAUNCHCHK();
                        continue;
                    }
                    int nchild = R.nbox[l];
                    int64_t n1 = (int64_t)nchild * 2 * R.nth[l - 1] * R.nph[l];
                    k_up_theta<T><<<nblocks(n1), WG, 0, stream_>>>(nchild, R.nth[l], R.nph[l], R.nth[l - 1], R.ipA[l],
                                                                   R.ipB[l], R.S[l], R.tmp);
                    LAUNCHCHK();
                    int64_t n2 = (int64_t)R.nbox[l - 1] * 2 * R.K[l - 1];
                    k_up_phi<T><<<nblocks(n2), WG, 0, stream_>>>(R.nbox[l - 1], R.nth[l - 1], R.nph[l - 1], R.nph[l],
                                                                 R.ipD[l], R.child_ptr[l - 1], R.child_idx[l - 1],
                                                                 R.slot[l], R.sup[l], R.tmp, R.S[l - 1]);
                    LAUNCHCHK();
                }
            }
            mark(3);
            for (Reg &R : regs_) {
                for (int l = 2; l <= f_; ++l) {
                    k_translate<T><<<nblocks((int64_t)R.nbox[l] * R.K[l]), WG, 0, stream_>>>(
                        R.nbox[l], R.K[l], R.il_ptr[l], R.il_src[l], R.il_off[l], R.trans[l], R.S[l], R.G[l]);
                    LAUNCHCHK();
                }
            }
            mark(4);
            for (Reg &R : regs_) {
                for (int l = 3; l <= f_; ++l) {
                    size_t lds = ((size_t)R.K[l - 1] + (size_t)R.nth[l - 1] * R.nph[l]) * sizeof(cx<T>);
                    if (lds <= LDS_LIMIT) {
                        k_dn_box<T><<<R.nbox[l], WG, lds, stream_>>>(R.nth[l], R.nph[l], R.nth[l - 1], R.nph[l - 1],
                                                                    R.ipA[l], R.ipB[l], R.ipD[l], R.parent[l], R.slot[l],
                                                                    R.sdn[l], R.G[l - 1], R.G[l]);
                        LAUNCHCHK();
                        continue;
                    }
                    int nchild = R.nbox[l];
                    int64_t n1 = (int64_t)nchild * 2 * R.nth[l - 1] * R.nph[l];
                    k_dn_phi<T><<<nblocks(n1), WG, 0, stream_>>>(nchild, R.nth[l - 1], R.nph[l - 1], R.nph[l], R.ipD[l],
                                                                 R.parent[l], R.slot[l], R.sdn[l], R.G[l - 1], R.tmp);
                    LAUNCHCHK();
                    int64_t n2 = (int64_t)nchild * 2 * R.K[l];
                    k_dn_theta<T><<<nblocks(n2), WG, 0, stream_>>>(nchild, R.nth[l], R.nph[l], R.nth[l - 1], R.ipA[l],
                                                                   R.ipB[l], R.tmp, R.G[l]);
                    LAUNCHCHK();
                }
            }
            mark(5);
            for (Reg &R : regs_) {
                const int f = f_;
                if (R.lossy)
                    k_receive<T, true><<<R.nbf, WG, 0, stream_>>>(R.K[f], R.edge_ptr, R.edge_pos, R.edge_sign, R.tx, R.rx,
                                                                  R.inv_et, R.G[f], y);
                else
                    k_receive<T, false><<<R.nbf, WG, 0, stream_>>>(R.K[f], R.edge_ptr, R.edge_pos, R.edge_sign, R.tx,
                                                                   nullptr, R.inv_et, R.G[f], y);
                LAUNCHCHK();
            }
        } else {
            mark(2); mark(3); mark(4); mark(5);
        }
        mark(6);
        if (profiling_) collect_matvec();
    }

    void ilu_internal(const cx<T> *v, cx<T> *z, cx<T> *w) {
        // ILU(0): forward z = L^-1 v colour by colour, backward w = U^-1 z in
        // reverse colour order.  Block-Jacobi: w = D^-1 v in one sweep.
        if (profiling_) HIPCHK(hipEventRecord(ev0_, stream_));
        size_t lds = (size_t)max_ilu_nc_ * 2 * sizeof(cx<T>);
        const bool use_lds = lds <= LDS_LIMIT;
        const unsigned groups = (unsigned)((2 * max_nrow_ + RW - 1) / RW);
        auto sweep = [&](int box0, int n, const int *cp, const int *cl, const int64_t *vp, const cx<T> *W,
                         const cx<T> *own, const cx<T> *other, cx<T> *out) {
            if (!n) return;
            dim3 grid(n, groups);
            if (use_lds)
                k_ilu<T, true><<<grid, RWG, lds, stream_>>>(box0, bstart_, cp, cl, vp, W, own, other, out);
            else
                k_ilu<T, false><<<grid, RWG, 0, stream_>>>(box0, bstart_, cp, cl, vp, W, own, other, out);
            LAUNCHCHK();
        };
        if (precond_ == SFMM_PRECOND_POLY) {
            // w = p(Z_near) v, product form over the Leja-ordered roots
            k_zero<T><<<nblocks(2 * ne_), WG, 0, stream_>>>(w, 2 * ne_);
            LAUNCHCHK();
            size_t lds_n = (size_t)max_ncol_ * 2 * sizeof(cx<T>);
            dim3 grid(nb_, (max_nrow_ + RW - 1) / RW);
            const cx<T> *cur = v;
            const int d = (int)inv_theta_.size();
            for (int k = 0; k < d; ++k) {
                cx<T> *next = (k % 2 == 0) ? z : pt_;
                const int last = (k == d - 1);
                if (lds_n <= LDS_LIMIT)
                    k_near<T, true, true><<<grid, RWG, lds_n, stream_>>>(bstart_, near_col_ptr_, near_cols_, near_val_ptr_,
                                                                        nA_, nB_, nC_, cur, next, w, inv_theta_[k], !last);
                else
                    k_near<T, false, true><<<grid, RWG, 0, stream_>>>(bstart_, near_col_ptr_, near_cols_, near_val_ptr_,
                                                                     nA_, nB_, nC_, cur, next, w, inv_theta_[k], !last);
                LAUNCHCHK();
                cur = next;
            }
        } else if (precond_ == SFMM_PRECOND_BLOCK_JACOBI) {
            sweep(0, nb_, fcol_ptr_, fcols_, fptr_, fval_, v, v, w);
        } else {
            for (int c = 0; c < 8; ++c)
                sweep(colour_ptr_[c], colour_ptr_[c + 1] - colour_ptr_[c], fcol_ptr_, fcols_, fptr_, fval_, v, z, z);
            for (int c = 7; c >= 0; --c)
                sweep(colour_ptr_[c], colour_ptr_[c + 1] - colour_ptr_[c], bcol_ptr_, bcols_, bptr_, bval_, z, w, w);
        }
        if (profiling_) {
            HIPCHK(hipEventRecord(ev1_, stream_));
            HIPCHK(hipEventSynchronize(ev1_));
            float ms = 0;
            HIPCHK(hipEventElapsedTime(&ms, ev0_, ev1_));
            times_.ms[6] += ms;
            times_.n[6] += 1;
        }
    }

    // ---- C ABI operations (boundary layout FP64 on device) ----
    void matvec(int n_rhs, const void *x_dev, void *y_dev, int parts) override {
        const int N = 2 * ne_;
        for (int r = 0; r < n_rhs; ++r) {
            const double2 *xb = (const double2 *)x_dev + (size_t)r * N;
            double2 *yb = (double2 *)y_dev + (size_t)r * N;
            k_to_internal<T><<<nblocks(ne_), WG, 0, stream_>>>(xb, pos_, ne_, xi_);
            LAUNCHCHK();
            matvec_internal(xi_, yi_, parts);
            k_to_boundary<T><<<nblocks(ne_), WG, 0, stream_>>>(yi_, pos_, ne_, yb);
            LAUNCHCHK();
        }
    }

    void precond(int n_rhs, const void *x_dev, void *y_dev) override {
        const int N = 2 * ne_;
        for (int r = 0; r < n_rhs; ++r) {
            const double2 *xb = (const double2 *)x_dev + (size_t)r * N;
            double2 *yb = (double2 *)y_dev + (size_t)r * N;
            k_to_internal<T><<<nblocks(ne_), WG, 0, stream_>>>(xb, pos_, ne_, xi_);
            LAUNCHCHK();
            const cx<T> *out = xi_;
            if (precond_ != SFMM_PRECOND_NONE) {
                ilu_internal(xi_, zi_, wi_);
                out = wi_;
            }
            k_to_boundary<T><<<nblocks(ne_), WG, 0, stream_>>>(out, pos_, ne_, yb);
            LAUNCHCHK();
        }
    }

    // FP64 internal helpers for GMRES
    // out = A M^-1 in (or A in, or M^-1 in); if zout is given, it receives
    // M^-1 in exactly as the product saw it (flexible GMRES keeps it).
    void op_apply(const double2 *in, double2 *out, bool precondition, bool product, double2 *zout = nullptr) {
        const int N = 2 * ne_;
        k_cast<double, T><<<nblocks(N), WG, 0, stream_>>>((const cx<double> *)in, xi_, N);
        LAUNCHCHK();
        const cx<T> *cur = xi_;
        if (precondition && precond_ != SFMM_PRECOND_NONE) {
            ilu_internal(xi_, zi_, wi_);
            cur = wi_;
        }
        if (zout) {
            k_cast<T, double><<<nblocks(N), WG, 0, stream_>>>(cur, (cx<double> *)zout, N);
            LAUNCHCHK();
        }
        if (product) {
            matvec_internal(cur, yi_, SFMM_PART_ALL);
            cur = yi_;
        }
        k_cast<T, double><<<nblocks(N), WG, 0, stream_>>>(cur, (cx<double> *)out, N);
        LAUNCHCHK();
    }

    double norm(const double2 *v) {
        const int N = 2 * ne_;
        k_norm2<<<red_blocks_, WG, 0, stream_>>>(v, N, dpart_);
        LAUNCHCHK();
        k_sum_real<<<1, 64, 0, stream_>>>(dpart_, red_blocks_, dscal_);
        LAUNCHCHK();
        double s = 0;
        copy_d2h(&s, dscal_, sizeof(double), stream_);
        return std::sqrt(s);
    }

    void solve(int n_rhs, const void *b_dev, void *x_dev, const void *x0_dev, int m, int max_iters, double tol,
               sfmm_solve_info *info, int verbose) override {
        const int N = 2 * ne_;
        ensure_krylov(m);
        bool all_ok = true;
        for (int r = 0; r < n_rhs; ++r) {
            auto t0 = std::chrono::steady_clock::now();
            const double2 *bb = (const double2 *)b_dev + (size_t)r * N;
            double2 *xb = (double2 *)x_dev + (size_t)r * N;
            k_perm_in<<<nblocks(ne_), WG, 0, stream_>>>(bb, pos_, ne_, kb_);
            LAUNCHCHK();
            if (x0_dev) {
                k_perm_in<<<nblocks(ne_), WG, 0, stream_>>>((const double2 *)x0_dev + (size_t)r * N, pos_, ne_, kx_);
            } else {
                HIPCHK(hipMemsetAsync(kx_, 0, sizeof(double2) * N, stream_));
            }
            LAUNCHCHK();
            const double nb = norm(kb_);
            int its = 0, restarts = 0;
            double rel = 0;
            bool converged = false;
            std::vector<cd> H((size_t)(m + 1) * m), g(m + 1), sn(m);
            std::vector<double> cs(m);
            if (nb == 0.0) {
                HIPCHK(hipMemsetAsync(kx_, 0, sizeof(double2) * N, stream_));
                converged = true;
            }
            bool first = true;
            while (!converged) {
                // r = b - A x   (skipped for a zero start)
                double2 *V0 = kV_;
                if (first && !x0_dev) {
                    HIPCHK(hipMemcpyAsync(V0, kb_, sizeof(double2) * N, hipMemcpyDeviceToDevice, stream_));
                } else {
                    op_apply(kx_, V0, false, true);
                    k_rsub<<<nblocks(N), WG, 0, stream_>>>(kb_, N, V0);
                    LAUNCHCHK();
                }
                first = false;
                double beta = norm(V0);
                rel = beta / nb;
                if (verbose >= 2)
                    std::fprintf(stderr, "sfmm gmres: rhs %d restart %d its %d true residual %.3e\n", r, restarts, its,
                                 rel);
                if (rel <= tol) {
                    converged = true;
                    break;
                }
                if (its >= max_iters) break;
                k_scale<<<nblocks(N), WG, 0, stream_>>>(V0, 1.0 / beta, N, V0);
                LAUNCHCHK();
                std::fill(g.begin(), g.end(), cd(0));
                g[0] = beta;
                int jend = 0;
                for (int j = 0; j < m; ++j) {
                    double2 *Vj = kV_ + (size_t)j * N;
                    double2 *w = kV_ + (size_t)(j + 1) * N;
                    op_apply(Vj, w, true, true, kZ_ + (size_t)j * N);
                    ++its;
                    // classical Gram-Schmidt, twice
                    std::vector<cd> h(j + 1, 0.0);
                    for (int pass = 0; pass < 2; ++pass) {
                        dim3 grid(red_blocks_, j + 1);
                        k_dots<<<grid, WG, 0, stream_>>>(kV_, N, N, w, dpartc_);
                        LAUNCHCHK();
                        k_sum_partials<<<j + 1, 64, 0, stream_>>>(dpartc_, red_blocks_, dh_);
                        LAUNCHCHK();
                        k_sub_vh<<<nblocks(N), WG, 0, stream_>>>(kV_, N, j + 1, N, dh_, w);
                        LAUNCHCHK();
                        std::vector<double2> hh(j + 1);
                        copy_d2h(hh.data(), dh_, sizeof(double2) * (j + 1), stream_);
                        for (int i = 0; i <= j; ++i) h[i] += cd(hh[i].x, hh[i].y);
                    }
                    double hn = norm(w);
                    for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = h[i];
                    H[(size_t)(j + 1) * m + j] = hn;
                    const bool breakdown = !(hn > 0);
                    if (!breakdown) {
                        k_scale<<<nblocks(N), WG, 0, stream_>>>(w, 1.0 / hn, N, w);
                        LAUNCHCHK();
                    }
                    for (int i = 0; i < j; ++i) {
                        cd a = H[(size_t)i * m + j], b2 = H[(size_t)(i + 1) * m + j];
                        H[(size_t)i * m + j] = cs[i] * a + sn[i] * b2;
                        H[(size_t)(i + 1) * m + j] = -std::conj(sn[i]) * a + cs[i] * b2;
                    }
                    {
                        cd a = H[(size_t)j * m + j], b2 = H[(size_t)(j + 1) * m + j];
                        double na = std::abs(a), nbb = std::abs(b2);
                        if (nbb == 0) {
                            cs[j] = 1;
                            sn[j] = 0;
                        } else if (na == 0) {
                            cs[j] = 0;
                            sn[j] = std::conj(b2) / nbb;
                        } else {
                            double rho = std::hypot(na, nbb);
                            cs[j] = na / rho;
                            sn[j] = (a / na) * std::conj(b2) / rho;
                        }
                        H[(size_t)j * m + j] = cs[j] * a + sn[j] * b2;
                        H[(size_t)(j + 1) * m + j] = 0;
                        g[j + 1] = -std::conj(sn[j]) * g[j];
                        g[j] = cs[j] * g[j];
                    }
                    jend = j + 1;
                    if (std::abs(g[j + 1]) / nb <= tol || its >= max_iters || breakdown) break;
                }
                // y = H^-1 g, x += M^-1 V y
                std::vector<cd> y(jend);
                for (int i = jend - 1; i >= 0; --i) {
                    cd s = g[i];
                    for (int l = i + 1; l < jend; ++l) s -= H[(size_t)i * m + l] * y[l];
                    y[i] = s / H[(size_t)i * m + i];
                }
                std::vector<double2> yd(jend);
                for (int i = 0; i < jend; ++i) yd[i] = make_double2(y[i].real(), y[i].imag());
                HIPCHK(hipMemcpyAsync(dh_, yd.data(), sizeof(double2) * jend, hipMemcpyHostToDevice, stream_));
                // flexible form: x += Z y with z_j = M^-1 v_j as used in the products
                k_lincomb<<<nblocks(N), WG, 0, stream_>>>(kZ_, N, jend, N, dh_, kt_);
                LAUNCHCHK();
                k_add<<<nblocks(N), WG, 0, stream_>>>(kt_, N, kx_);
                LAUNCHCHK();
                ++restarts;
            }
            k_perm_out<<<nblocks(ne_), WG, 0, stream_>>>(kx_, pos_, ne_, xb);
            LAUNCHCHK();
            HIPCHK(hipStreamSynchronize(stream_));
            double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            if (info) {
                info[r].converged = converged ? 1 : 0;
                info[r].iterations = its;
                info[r].restarts = restarts;
                info[r].true_residual = rel;
                info[r].seconds = secs;
            }
            all_ok = all_ok && converged;
        }
        if (!all_ok) throw Error(SFMM_E_NOT_CONVERGED, "GMRES did not reach the tolerance within max_iters");
    }

    void planewave_rhs(int n_rhs, const double *angles, const double *pol, void *b_dev) override {
        const int N = 2 * ne_;
        std::vector<cd> b(N);
        for (int r = 0; r < n_rhs; ++r) {
            sfmm::planewave_rhs(h_.mesh, angles[2 * r], angles[2 * r + 1], pol ? pol[r] : 1.0, b.data());
            copy_h2d((double2 *)b_dev + (size_t)r * N, b.data(), sizeof(cd) * N, stream_);
        }
        HIPCHK(hipStreamSynchronize(stream_));
    }

    void rcs(int n_rhs, const void *x_dev, int n_dirs, const double *tp, double *sigma) override {
        const int N = 2 * ne_;
        std::vector<cd> x(N);
        for (int r = 0; r < n_rhs; ++r) {
            copy_d2h(x.data(), (const double2 *)x_dev + (size_t)r * N, sizeof(cd) * N, stream_);
            for (int d = 0; d < n_dirs; ++d) {
                cd Ft, Fp;
                far_field(h_.mesh, x.data(), tp[2 * d], tp[2 * d + 1], &Ft, &Fp);
                sigma[((size_t)r * n_dirs + d) * 2] = 4 * PI * std::norm(Ft);
                sigma[((size_t)r * n_dirs + d) * 2 + 1] = 4 * PI * std::norm(Fp);
            }
        }
    }

  private:
    struct Reg {
        cx<T> et{}, inv_et{};
        bool lossy = false;
        int nbf = 0;
        int *edge_ptr = nullptr, *edge_pos = nullptr, *edge_sign = nullptr;
        cx<T> *tx = nullptr, *rx = nullptr, *tmp = nullptr;
        int K[MAXLEV] = {0}, nth[MAXLEV] = {0}, nph[MAXLEV] = {0}, nbox[MAXLEV] = {0};
        cx<T> *S[MAXLEV] = {nullptr}, *G[MAXLEV] = {nullptr}, *trans[MAXLEV] = {nullptr};
        int *il_ptr[MAXLEV] = {nullptr}, *il_src[MAXLEV] = {nullptr}, *il_off[MAXLEV] = {nullptr};
        int *parent[MAXLEV] = {nullptr}, *slot[MAXLEV] = {nullptr};
        int *child_ptr[MAXLEV] = {nullptr}, *child_idx[MAXLEV] = {nullptr};
        T *ipA[MAXLEV] = {nullptr}, *ipB[MAXLEV] = {nullptr}, *ipD[MAXLEV] = {nullptr}, *ipDt[MAXLEV] = {nullptr};
        cx<T> *sup[MAXLEV] = {nullptr}, *sdn[MAXLEV] = {nullptr};
    };

    template <typename U>
    U *upload(const std::vector<U> &v) {
        U *p = (U *)device_alloc(sizeof(U) * std::max<size_t>(v.size(), 1));
        allocs_.push_back(p);
        bytes_ += sizeof(U) * v.size();
        if (!v.empty()) HIPCHK(hipMemcpy(p, v.data(), sizeof(U) * v.size(), hipMemcpyHostToDevice));
        return p;
    }
    cx<T> *upload_cx(const std::vector<cd> &v) {
        std::vector<cx<T>> t(v.size());
        for (size_t i = 0; i < v.size(); ++i) t[i] = to_cx<T>(v[i]);
        return upload(t);
    }
    T *upload_real(const std::vector<double> &v) {
        std::vector<T> t(v.begin(), v.end());
        return upload(t);
    }
    cx<T> *alloc_cx(size_t n) {
        cx<T> *p = (cx<T> *)device_alloc(sizeof(cx<T>) * std::max<size_t>(n, 1));
        allocs_.push_back(p);
        bytes_ += sizeof(cx<T>) * n;
        return p;
    }
    template <typename U>
    U *alloc_raw(size_t n) {
        U *p = (U *)device_alloc(sizeof(U) * std::max<size_t>(n, 1));
        allocs_.push_back(p);
        bytes_ += sizeof(U) * n;
        return p;
    }

    void ensure_krylov(int m) {
        const int N = 2 * ne_;
        if (m <= kM_) return;
        kM_ = m;
        kV_ = alloc_raw<double2>((size_t)(m + 1) * N);
        kZ_ = alloc_raw<double2>((size_t)m * N);
        kb_ = alloc_raw<double2>(N);
        kx_ = alloc_raw<double2>(N);
        ku_ = alloc_raw<double2>(N);
        kt_ = alloc_raw<double2>(N);
        red_blocks_ = std::min(256, (int)nblocks(N, WG * 4));
        dpartc_ = alloc_raw<double2>((size_t)(m + 1) * red_blocks_);
        dpart_ = alloc_raw<double>(red_blocks_);
        dh_ = alloc_raw<double2>(m + 1);
        dscal_ = alloc_raw<double>(1);
    }

    void mark(int i) {
        if (profiling_) HIPCHK(hipEventRecord(evs_[i], stream_));
    }
    void collect_matvec() {
        HIPCHK(hipEventSynchronize(evs_[6]));
        float ms;
        for (int i = 0; i < 6; ++i) {
            HIPCHK(hipEventElapsedTime(&ms, evs_[i], evs_[i + 1]));
            times_.ms[i] += ms;
            times_.n[i] += 1;
        }
        HIPCHK(hipEventElapsedTime(&ms, evs_[0], evs_[6]));
        times_.ms[7] += ms;
        times_.n[7] += 1;
    }

    const BodyHost &h_;
    int dev_;
    hipStream_t stream_;
    int ne_ = 0, nb_ = 0, f_ = 0;
    std::array<int, 9> colour_ptr_{};
    int *pos_ = nullptr, *bstart_ = nullptr;
    int *near_col_ptr_ = nullptr, *near_cols_ = nullptr;
    int64_t *near_val_ptr_ = nullptr;
    cx<T> *nA_ = nullptr, *nB_ = nullptr, *nC_ = nullptr;
    int max_ncol_ = 0, max_nrow_ = 0, max_ilu_nc_ = 0, precond_ = SFMM_PRECOND_ILU0;
    int *fcol_ptr_ = nullptr, *fcols_ = nullptr, *bcol_ptr_ = nullptr, *bcols_ = nullptr;
    int64_t *fptr_ = nullptr, *bptr_ = nullptr;
    cx<T> *fval_ = nullptr, *bval_ = nullptr;
    std::vector<Reg> regs_;
    cx<T> *xi_ = nullptr, *yi_ = nullptr, *zi_ = nullptr, *wi_ = nullptr, *pt_ = nullptr;
    std::vector<cx<T>> inv_theta_;
    // Krylov workspace
    int kM_ = 0, red_blocks_ = 1;
    double2 *kV_ = nullptr, *kZ_ = nullptr, *kb_ = nullptr, *kx_ = nullptr, *ku_ = nullptr, *kt_ = nullptr;
    double2 *dpartc_ = nullptr, *dh_ = nullptr;
    double *dpart_ = nullptr, *dscal_ = nullptr;
    std::vector<void *> allocs_;
    int64_t bytes_ = 0;
    bool profiling_ = false;
    hipEvent_t ev0_ = nullptr, ev1_ = nullptr;
    hipEvent_t evs_[7] = {nullptr};
    StageTimes times_;
};

}  // namespace

std::unique_ptr<DeviceBody> make_device_body(const BodyHost &h, int precision, int device, void *stream) {
    check_device(device);
    if (precision == SFMM_PREC_FP64) return std::make_unique<DeviceBodyT<double>>(h, device, stream);
    if (precision == SFMM_PREC_FP32) return std::make_unique<DeviceBodyT<float>>(h, device, stream);
    throw Error(SFMM_E_UNSUPPORTED, "precision mode not implemented yet");
}

}  // namespace sfmm
