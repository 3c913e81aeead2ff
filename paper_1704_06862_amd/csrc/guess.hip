// Learned initial guess for GMRES (an addition to the paper's method): a
// network trained on the device, with hand-written kernels, on currents the
// solver produced for other incidence angles.
//
//   POD basis   U = first r left singular vectors of X = [x_1 .. x_n]
//               (Gram matrix X^H X on the device, Hermitian Jacobi
//               eigen-decomposition on the host, U = X V Sigma^-1)
//   features    the far field of the right-hand side b read as surface
//               currents, on a coarse theta/phi grid (Re/Im of the theta
//               and phi components, FP64, divided by ||b|| and scaled by one
//               scalar), after cos/sin(m theta), cos/sin(m phi), m = 1..M
//   network     y = Ws^T z_p + MLP(z) / s_r: a linear path from the pattern
//               features, the minimum-norm least-squares fit of the scaled
//               POD coefficients (FP64), and two tanh hidden layers trained
//               by Adam on what the linear path leaves, scaled to unit RMS
//   arithmetic  MLP GEMMs on the matrix cores with bf16-split operands
//               (hi + lo, three v_mfma_f32_16x16x32_bf16 per K step, FP32
//               accumulation), FP32 master weights and optimizer state; the
//               linear path in FP64
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "guess.hpp"

namespace sfmm {

#define GHIPCHK(expr)                                                                            \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            throw Error(SFMM_E_DEVICE, std::string(#expr) + " failed: " + hipGetErrorString(e_)); \
    } while (0)

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// C[i][j] = act( sum_k A(i,k) B(k,j) + bias[j] ), A(i,k) = A[i*a0 + k*a1],
// B(k,j) = B[k*b0 + j*b1], C row-major with ldc; FP32 operands split into
// bf16 hi + lo, hi*hi + hi*lo + lo*hi on v_mfma_f32_16x16x32_bf16.  One wave
// per 32 x 32 block of C (2 x 2 MFMA tiles).  Lane l of a 16 x 16 tile holds
// A row l % 16 / B column l % 16 at K indices 8 (l / 16) .. + 7 and receives
// D rows 4 (l / 16) .. + 3 of column l % 16.
__global__ void __launch_bounds__(64) k_gemm_mma(int M, int N, int K, const float *__restrict__ A, int64_t a0,
                                                 int64_t a1, const float *__restrict__ B, int64_t b0, int64_t b1,
                                                 const float *__restrict__ bias, int act, float *__restrict__ C,
                                                 int64_t ldc) {
    const int l = threadIdx.x, i0 = blockIdx.y * 32, j0 = blockIdx.x * 32;
    const int lr = l & 15, lk = (l >> 4) * 8;
    f32x4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += 32) {
        bf16x8 ah[2], al[2], bh[2], bl[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const int i = i0 + 16 * t + lr, j = j0 + 16 * t + lr;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int k = k0 + lk + e;
                const float va = (i < M && k < K) ? A[i * a0 + k * a1] : 0.f;
                const float vb = (j < N && k < K) ? B[k * b0 + j * b1] : 0.f;
                const __bf16 ha = (__bf16)va, hb = (__bf16)vb;
                ah[t][e] = ha;
                al[t][e] = (__bf16)(va - (float)ha);
                bh[t][e] = hb;
                bl[t][e] = (__bf16)(vb - (float)hb);
            }
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[a], bh[b], acc[a][b], 0, 0, 0);
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bl[b], acc[a][b], 0, 0, 0);
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bh[b], acc[a][b], 0, 0, 0);
            }
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int j = j0 + 16 * b + lr;
            if (j >= N) continue;
            const float bj = bias ? bias[j] : 0.f;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = i0 + 16 * a + (l >> 4) * 4 + v;
                if (i >= M) continue;
                float c = acc[a][b][v] + bj;
                if (act == 1) c = tanhf(c);
                C[i * ldc + j] = c;
            }
        }
}

// FP64: C[i][j] = sum_k A(i,k) B(k,j), strides as k_gemm_mma, 16 x 16 tiles
// through LDS
constexpr int DT = 16;
__global__ void __launch_bounds__(DT *DT) k_dgemm(int M, int N, int K, const double *__restrict__ A, int64_t a0,
                                                  int64_t a1, const double *__restrict__ B, int64_t b0, int64_t b1,
                                                  double *__restrict__ C, int64_t ldc) {
    __shared__ double As[DT][DT + 1], Bs[DT][DT + 1];
    const int ti = threadIdx.x / DT, tj = threadIdx.x % DT;
    const int i = blockIdx.y * DT + ti, j = blockIdx.x * DT + tj;
    double acc = 0.0;
    for (int k0 = 0; k0 < K; k0 += DT) {
        const int ka = k0 + tj, kb = k0 + ti;
        As[ti][tj] = (i < M && ka < K) ? A[i * a0 + ka * a1] : 0.0;
        Bs[ti][tj] = (kb < K && j < N) ? B[kb * b0 + j * b1] : 0.0;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < DT; ++k) acc += As[ti][k] * Bs[k][tj];
        __syncthreads();
    }
    if (i < M && j < N) C[i * ldc + j] = acc;
}

// delta *= (1 - h^2)
__global__ void k_tanh_back(int n, const float *__restrict__ h, float *__restrict__ d) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] *= 1.f - h[i] * h[i];
}

// diff = (out - Y) / B ; per-block partial of 0.5 sum (out - Y)^2
__global__ void k_mse(int n, float invB, const float *__restrict__ out, const float *__restrict__ Y,
                      float *__restrict__ diff, double *__restrict__ partial) {
    __shared__ double red[256];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double s = 0;
    if (i < n) {
        const float d = out[i] - Y[i];
        diff[i] = d * invB;
        s = 0.5 * (double)d * d;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// db[j] = sum_i d[i][j]
__global__ void k_colsum(int rows, int cols, const float *__restrict__ d, float *__restrict__ db) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= cols) return;
    float s = 0.f;
    for (int i = 0; i < rows; ++i) s += d[(int64_t)i * cols + j];
    db[j] = s;
}

__global__ void k_adam(int64_t n, float lr, float b1, float b2, float eps, float c1, float c2,
                       const float *__restrict__ g, float *__restrict__ m, float *__restrict__ v,
                       float *__restrict__ p) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Adam step whose step count lives on the device (so that a captured graph
// can replay it): t = *step + 1, step size lr0 (1 + cos(pi (t - 1) / E)) / 2
// for t <= E, bias corrections 1 - b^t.
__global__ void k_adam_sched(int64_t n, float lr0, int E, float b1, float b2, float eps,
                             const int *__restrict__ step, const float *__restrict__ g, float *__restrict__ m,
                             float *__restrict__ v, float *__restrict__ p) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int t = *step + 1;
    const float lr = lr0 * 0.5f * (1.f + cosf(3.14159265358979f * (float)(t - 1) / (float)E));
    const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void k_step_inc(int *step) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *step += 1;
}

inline unsigned nb(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

void gemm(hipStream_t s, int M, int N, int K, const float *A, int64_t a0, int64_t a1, const float *B, int64_t b0,
          int64_t b1, const float *bias, int act, float *C, int64_t ldc) {
    dim3 grid(nb(N, 32), nb(M, 32));
    k_gemm_mma<<<grid, 64, 0, s>>>(M, N, K, A, a0, a1, B, b0, b1, bias, act, C, ldc);
    GHIPCHK(hipGetLastError());
}

void dgemm(hipStream_t s, int M, int N, int K, const double *A, int64_t a0, int64_t a1, const double *B,
           int64_t b0, int64_t b1, double *C, int64_t ldc) {
    dim3 grid(nb(N, DT), nb(M, DT));
    k_dgemm<<<grid, DT * DT, 0, s>>>(M, N, K, A, a0, a1, B, b0, b1, C, ldc);
    GHIPCHK(hipGetLastError());
}

}  // namespace

void use_device(int device) { GHIPCHK(hipSetDevice(device)); }

int64_t mlp_param_count(const std::vector<int> &sizes) {
    int64_t n = 0;
    for (size_t l = 0; l + 1 < sizes.size(); ++l) n += (int64_t)sizes[l] * sizes[l + 1] + sizes[l + 1];
    return n;
}

Mlp::Mlp(const std::vector<int> &sizes, void *stream) : sizes_(sizes), stream_(stream) {
    if (sizes.size() < 2) throw Error(SFMM_E_INVALID_ARG, "MLP needs at least two layer sizes");
    for (int s : sizes)
        if (s <= 0 || s > 65536) throw Error(SFMM_E_INVALID_ARG, "bad MLP layer size");
    np_ = mlp_param_count(sizes);
    GHIPCHK(hipMalloc(&p_, sizeof(float) * np_));
    GHIPCHK(hipMalloc(&g_, sizeof(float) * np_));
    GHIPCHK(hipMalloc(&m_, sizeof(float) * np_));
    GHIPCHK(hipMalloc(&v_, sizeof(float) * np_));
    GHIPCHK(hipMemsetAsync(m_, 0, sizeof(float) * np_, (hipStream_t)stream_));
    GHIPCHK(hipMemsetAsync(v_, 0, sizeof(float) * np_, (hipStream_t)stream_));
}

Mlp::~Mlp() {
    for (float *q : {p_, g_, m_, v_}) (void)hipFree(q);
    for (float *q : acts_) (void)hipFree(q);
    (void)hipFree(delta_);
    (void)hipFree(delta2_);
    (void)hipFree(partial_);
}

void Mlp::set_params(const float *host) {
    GHIPCHK(hipMemcpyAsync(p_, host, sizeof(float) * np_, hipMemcpyHostToDevice, (hipStream_t)stream_));
    GHIPCHK(hipStreamSynchronize((hipStream_t)stream_));
}
void Mlp::get_params(float *host) const {
    GHIPCHK(hipMemcpyAsync(host, p_, sizeof(float) * np_, hipMemcpyDeviceToHost, (hipStream_t)stream_));
    GHIPCHK(hipStreamSynchronize((hipStream_t)stream_));
}
void Mlp::get_grads(float *host) const {
    GHIPCHK(hipMemcpyAsync(host, g_, sizeof(float) * np_, hipMemcpyDeviceToHost, (hipStream_t)stream_));
    GHIPCHK(hipStreamSynchronize((hipStream_t)stream_));
}

void Mlp::init_uniform(uint64_t seed, bool zero_last) {
    // SplitMix64 (Steele, Lea, Flood 2014) -> uniform [0,1); weights
    // U(-sqrt(6/(in+out)), +sqrt(6/(in+out))), biases zero; with zero_last
    // the output layer starts at zero
    std::vector<float> h(np_, 0.f);
    uint64_t state = seed;
    auto next = [&]() {
        uint64_t z = (state += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        return (double)(z >> 11) * (1.0 / 9007199254740992.0);
    };
    int64_t off = 0;
    for (size_t l = 0; l + 1 < sizes_.size(); ++l) {
        const int a = sizes_[l], b = sizes_[l + 1];
        const double lim = std::sqrt(6.0 / (a + b));
        const bool zero = zero_last && l + 2 == sizes_.size();
        for (int64_t q = 0; q < (int64_t)a * b; ++q) h[off + q] = zero ? 0.f : (float)((2.0 * next() - 1.0) * lim);
        off += (int64_t)a * b + b;
    }
    set_params(h.data());
    GHIPCHK(hipMemsetAsync(m_, 0, sizeof(float) * np_, (hipStream_t)stream_));
    GHIPCHK(hipMemsetAsync(v_, 0, sizeof(float) * np_, (hipStream_t)stream_));
    t_ = 0;
}

void Mlp::ensure_batch(int B) {
    if (B <= cap_) return;
    for (float *q : acts_) (void)hipFree(q);
    acts_.assign(sizes_.size(), nullptr);
    int wmax = 0;
    for (size_t l = 0; l < sizes_.size(); ++l) {
        GHIPCHK(hipMalloc(&acts_[l], sizeof(float) * (size_t)B * sizes_[l]));
        wmax = std::max(wmax, sizes_[l]);
    }
    (void)hipFree(delta_);
    (void)hipFree(delta2_);
    (void)hipFree(partial_);
    GHIPCHK(hipMalloc(&delta_, sizeof(float) * (size_t)B * wmax));
    GHIPCHK(hipMalloc(&delta2_, sizeof(float) * (size_t)B * wmax));
    GHIPCHK(hipMalloc(&partial_, sizeof(double) * (nb((int64_t)B * sizes_.back(), 256) + 1)));
    cap_ = B;
}

const float *Mlp::forward(int B, const float *X) {
    ensure_batch(B);
    hipStream_t s = (hipStream_t)stream_;
    GHIPCHK(hipMemcpyAsync(acts_[0], X, sizeof(float) * (size_t)B * sizes_[0], hipMemcpyDeviceToDevice, s));
    int64_t off = 0;
    const int L = (int)sizes_.size() - 1;
    for (int l = 0; l < L; ++l) {
        const int a = sizes_[l], b = sizes_[l + 1];
        const float *W = p_ + off, *bias = p_ + off + (int64_t)a * b;
        gemm(s, B, b, a, acts_[l], a, 1, W, b, 1, bias, l < L - 1 ? 1 : 0, acts_[l + 1], b);
        off += (int64_t)a * b + b;
    }
    return acts_[L];
}

double Mlp::loss_grad(int B, const float *X, const float *Y, bool want_loss) {
    hipStream_t s = (hipStream_t)stream_;
    const float *out = forward(B, X);
    const int L = (int)sizes_.size() - 1;
    const int O = sizes_[L];
    const int64_t n = (int64_t)B * O;
    const unsigned nbk = nb(n, 256);
    k_mse<<<nbk, 256, 0, s>>>((int)n, 1.f / B, out, Y, delta_, partial_);
    GHIPCHK(hipGetLastError());
    // offsets of each layer
    std::vector<int64_t> offs(L + 1, 0);
    for (int l = 0; l < L; ++l) offs[l + 1] = offs[l] + (int64_t)sizes_[l] * sizes_[l + 1] + sizes_[l + 1];
    float *d = delta_, *dn = delta2_;
    for (int l = L - 1; l >= 0; --l) {
        const int a = sizes_[l], b = sizes_[l + 1];
        float *gW = g_ + offs[l], *gb = g_ + offs[l] + (int64_t)a * b;
        const float *W = p_ + offs[l];
        // dW = acts[l]^T d  (a x b), K = batch
        gemm(s, a, b, B, acts_[l], 1, a, d, b, 1, nullptr, 0, gW, b);
        k_colsum<<<nb(b, 256), 256, 0, s>>>(B, b, d, gb);
        GHIPCHK(hipGetLastError());
        if (l > 0) {
            // dn = d W^T (B x a), then times tanh'
            gemm(s, B, a, b, d, b, 1, W, 1, b, nullptr, 0, dn, a);
            k_tanh_back<<<nb((int64_t)B * a, 256), 256, 0, s>>>(B * a, acts_[l], dn);
            GHIPCHK(hipGetLastError());
            std::swap(d, dn);
        }
    }
    if (!want_loss) return std::nan("");
    std::vector<double> part(nbk);
    GHIPCHK(hipMemcpyAsync(part.data(), partial_, sizeof(double) * nbk, hipMemcpyDeviceToHost, s));
    GHIPCHK(hipStreamSynchronize(s));
    double loss = 0;
    for (double v : part) loss += v;
    return loss / B;
}

void Mlp::adam_scheduled(const int *step, double lr0, int epochs, double b1, double b2, double eps) {
    k_adam_sched<<<nb(np_, 256), 256, 0, (hipStream_t)stream_>>>(np_, (float)lr0, epochs, (float)b1, (float)b2,
                                                                 (float)eps, step, g_, m_, v_, p_);
    GHIPCHK(hipGetLastError());
    k_step_inc<<<1, 64, 0, (hipStream_t)stream_>>>(const_cast<int *>(step));
    GHIPCHK(hipGetLastError());
}

void Mlp::adam_step(double lr, double b1, double b2, double eps) {
    ++t_;
    const double c1 = 1.0 - std::pow(b1, t_), c2 = 1.0 - std::pow(b2, t_);
    k_adam<<<nb(np_, 256), 256, 0, (hipStream_t)stream_>>>(np_, (float)lr, (float)b1, (float)b2, (float)eps,
                                                           (float)c1, (float)c2, g_, m_, v_, p_);
    GHIPCHK(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Hermitian eigen-decomposition (cyclic Jacobi), host, small n.
void hermitian_eig(int n, std::vector<cd> &A, std::vector<double> &w, std::vector<cd> &V) {
    V.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
    auto a = [&](int i, int j) -> cd & { return A[(size_t)i * n + j]; };
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0, tot = 0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                tot += std::norm(a(i, j));
                if (i != j) off += std::norm(a(i, j));
            }
        if (off <= 1e-30 * tot) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                const cd apq = a(p, q);
                const double mag = std::abs(apq);
                if (mag == 0) continue;
                // rotation that annihilates a(p,q) of the Hermitian 2x2 block
                const double app = a(p, p).real(), aqq = a(q, q).real();
                const cd ph = apq / mag;                       // e^{j alpha}
                const double theta = 0.5 * std::atan2(2.0 * mag, aqq - app);
                const double c = std::cos(theta), s = std::sin(theta);
                // columns: [p q] <- [p q] [[c, s ph], [-s conj(ph), c]]
                for (int i = 0; i < n; ++i) {
                    const cd xp = a(i, p), xq = a(i, q);
                    a(i, p) = c * xp - s * std::conj(ph) * xq;
                    a(i, q) = s * ph * xp + c * xq;
                }
                for (int j = 0; j < n; ++j) {
                    const cd xp = a(p, j), xq = a(q, j);
                    a(p, j) = c * xp - s * ph * xq;
                    a(q, j) = s * std::conj(ph) * xp + c * xq;
                }
                for (int i = 0; i < n; ++i) {
                    const cd vp = V[(size_t)i * n + p], vq = V[(size_t)i * n + q];
                    V[(size_t)i * n + p] = c * vp - s * std::conj(ph) * vq;
                    V[(size_t)i * n + q] = s * ph * vp + c * vq;
                }
            }
    }
    w.resize(n);
    for (int i = 0; i < n; ++i) w[i] = a(i, i).real();
}

}  // namespace sfmm

namespace sfmm {

namespace {

// partial[(i * nbv + j) * gridDim.x + blk] = sum over chunk of conj(a_i) b_j
__global__ void __launch_bounds__(256) k_cross_dots(const double2 *__restrict__ A, int64_t lda,
                                                    const double2 *__restrict__ B, int64_t ldb, int nbv, int N,
                                                    int diag, double2 *__restrict__ partial) {
    __shared__ double2 red[256];
    const int i = blockIdx.y, j = blockIdx.z;
    const double2 *a = A + (int64_t)i * lda, *b = B + (int64_t)(diag ? i : j) * ldb;
    double sx = 0, sy = 0;
    for (int q = blockIdx.x * 256 + threadIdx.x; q < N; q += gridDim.x * 256) {
        const double2 u = a[q], v = b[q];
        sx += u.x * v.x + u.y * v.y;
        sy += u.x * v.y - u.y * v.x;
    }
    red[threadIdx.x] = make_double2(sx, sy);
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            red[threadIdx.x].x += red[threadIdx.x + o].x;
            red[threadIdx.x].y += red[threadIdx.x + o].y;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[((int64_t)i * nbv + j) * gridDim.x + blockIdx.x] = red[0];
}

__global__ void k_lincomb_set(const double2 *__restrict__ V, int64_t ld, int nv, const double2 *__restrict__ coef,
                              int N, double2 *__restrict__ out, int64_t ldo) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x, s = blockIdx.y;
    if (q >= N) return;
    double2 acc = make_double2(0, 0);
    for (int j = 0; j < nv; ++j) {
        const double2 v = V[(int64_t)j * ld + q], c = coef[(int64_t)s * nv + j];
        acc.x += v.x * c.x - v.y * c.y;
        acc.y += v.x * c.y + v.y * c.x;
    }
    out[(int64_t)s * ldo + q] = acc;
}

}  // namespace

namespace {

void dots_impl(const void *A, int64_t lda, int na, const void *B, int64_t ldb, int nbv, int N, int diag,
               cd *out_host, void *stream) {
    hipStream_t s = (hipStream_t)stream;
    const int nblk = 16;
    double2 *partial = nullptr;
    GHIPCHK(hipMalloc(&partial, sizeof(double2) * (size_t)na * nbv * nblk));
    k_cross_dots<<<dim3(nblk, na, nbv), 256, 0, s>>>((const double2 *)A, lda, (const double2 *)B, ldb, nbv, N,
                                                     diag, partial);
    GHIPCHK(hipGetLastError());
    std::vector<double2> h((size_t)na * nbv * nblk);
    GHIPCHK(hipMemcpyAsync(h.data(), partial, sizeof(double2) * h.size(), hipMemcpyDeviceToHost, s));
    GHIPCHK(hipStreamSynchronize(s));
    (void)hipFree(partial);
    for (int64_t q = 0; q < (int64_t)na * nbv; ++q) {
        cd acc = 0;
        for (int b = 0; b < nblk; ++b) acc += cd(h[q * nblk + b].x, h[q * nblk + b].y);
        out_host[q] = acc;
    }
}

}  // namespace

void cross_dots(const void *A, int64_t lda, int na, const void *B, int64_t ldb, int nbv, int N, cd *out_host,
                void *stream) {
    dots_impl(A, lda, na, B, ldb, nbv, N, 0, out_host, stream);
}

void self_norms(const void *A, int64_t lda, int n, int N, double *out_host, void *stream) {
    std::vector<cd> d(n);
    dots_impl(A, lda, n, A, lda, 1, N, 1, d.data(), stream);
    for (int i = 0; i < n; ++i) out_host[i] = std::sqrt(std::max(d[i].real(), 0.0));
}

void lincomb(const void *vecs, int64_t ld, int nv, const cd *coef_host, int ns, int N, void *out, int64_t ldo,
             void *stream) {
    hipStream_t s = (hipStream_t)stream;
    double2 *coef = nullptr;
    GHIPCHK(hipMalloc(&coef, sizeof(double2) * (size_t)ns * nv));
    GHIPCHK(hipMemcpyAsync(coef, coef_host, sizeof(double2) * (size_t)ns * nv, hipMemcpyHostToDevice, s));
    k_lincomb_set<<<dim3((N + 255) / 256, ns), 256, 0, s>>>((const double2 *)vecs, ld, nv, coef, N, (double2 *)out,
                                                            ldo);
    GHIPCHK(hipGetLastError());
    GHIPCHK(hipStreamSynchronize(s));
    (void)hipFree(coef);
}

}  // namespace sfmm

namespace sfmm {

Guess::~Guess() {
    (void)hipFree(U_);
    (void)hipFree(W_);
    (void)hipFree(Ws_);
}

void Guess::span_predict(int n, const void *B, void *X0,
                         const std::function<void(int, const void *, void *)> &product) {
    if (!U_) throw Error(SFMM_E_INVALID_ARG, "learned guess is not trained (call sfmm_guess_fit first)");
    if (n < 1) throw Error(SFMM_E_INVALID_ARG, "n must be positive");
    const int r = r_;
    if (!W_) {
        GHIPCHK(hipMalloc(&W_, sizeof(double2) * (size_t)r * N_));
        product(r, U_, W_);
        gram_.assign((size_t)r * r, 0.0);
        cross_dots(W_, N_, r, W_, N_, r, N_, gram_.data(), stream_);
    }
    // c_s = (W^H W)^-1 W^H b_s: Gaussian elimination with partial pivoting
    std::vector<cd> h((size_t)r * n);
    cross_dots(W_, N_, r, B, N_, n, N_, h.data(), stream_);   // h[k][s] = w_k^H b_s
    std::vector<cd> A = gram_, coef((size_t)n * r);
    std::vector<cd> rhs(h);
    for (int k = 0; k < r; ++k) {
        int piv = k;
        for (int i = k + 1; i < r; ++i)
            if (std::abs(A[(size_t)i * r + k]) > std::abs(A[(size_t)piv * r + k])) piv = i;
        if (piv != k) {
            for (int j = 0; j < r; ++j) std::swap(A[(size_t)k * r + j], A[(size_t)piv * r + j]);
            for (int s2 = 0; s2 < n; ++s2) std::swap(rhs[(size_t)k * n + s2], rhs[(size_t)piv * n + s2]);
        }
        const cd p = A[(size_t)k * r + k];
        if (!(std::abs(p) > 0)) throw Error(SFMM_E_BREAKDOWN, "singular reduced system in the span guess");
        for (int i = k + 1; i < r; ++i) {
            const cd f = A[(size_t)i * r + k] / p;
            for (int j = k; j < r; ++j) A[(size_t)i * r + j] -= f * A[(size_t)k * r + j];
            for (int s2 = 0; s2 < n; ++s2) rhs[(size_t)i * n + s2] -= f * rhs[(size_t)k * n + s2];
        }
    }
    for (int s2 = 0; s2 < n; ++s2)
        for (int i = r - 1; i >= 0; --i) {
            cd v = rhs[(size_t)i * n + s2];
            for (int j = i + 1; j < r; ++j) v -= A[(size_t)i * r + j] * coef[(size_t)s2 * r + j];
            coef[(size_t)s2 * r + i] = v / A[(size_t)i * r + i];
        }
    lincomb(U_, N_, r, coef.data(), n, N_, X0, N_, stream_);
}

void Guess::set_stream(void *s) {
    stream_ = s;
    if (net_) net_->set_stream(s);
}

namespace {

// device buffer freed at scope exit
template <typename T>
struct DevBuf {
    T *p = nullptr;
    explicit DevBuf(size_t n) { GHIPCHK(hipMalloc(&p, sizeof(T) * std::max<size_t>(n, 1))); }
    ~DevBuf() { (void)hipFree(p); }
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
};

}  // namespace

void Guess::features(int n, const double *angles, const void *B, std::vector<float> &Z, std::vector<double> &Zp,
                     std::vector<double> &nb, bool set_scale) {
    constexpr double kPi = 3.14159265358979323846;
    hipStream_t st = (hipStream_t)stream_;
    const int M = o_.harmonics, nt = o_.n_theta, nph = o_.n_phi, nd = nt * nph, np = 4 * nd, nf = 4 * M + np;
    // coarse direction grid: theta at the midpoints of nt bands, phi uniform
    std::vector<double> dirs(2 * (size_t)nd);
    for (int i = 0; i < nt; ++i)
        for (int j = 0; j < nph; ++j) {
            dirs[2 * ((size_t)i * nph + j)] = (i + 0.5) * kPi / nt;
            dirs[2 * ((size_t)i * nph + j) + 1] = j * 2.0 * kPi / nph;
        }
    DevBuf<double> dd(dirs.size()), dF((size_t)n * np);
    GHIPCHK(hipMemcpyAsync(dd.p, dirs.data(), sizeof(double) * dirs.size(), hipMemcpyHostToDevice, st));
    pattern_(n, B, nd, dd.p, dF.p);
    Zp.assign((size_t)n * np, 0.0);
    GHIPCHK(hipMemcpyAsync(Zp.data(), dF.p, sizeof(double) * Zp.size(), hipMemcpyDeviceToHost, st));
    nb.assign(n, 0.0);
    self_norms(B, N_, n, N_, nb.data(), stream_);   // synchronises the stream
    for (int s = 0; s < n; ++s) {
        const double inv = nb[s] > 0 ? 1.0 / nb[s] : 0.0;
        for (int q = 0; q < np; ++q) Zp[(size_t)s * np + q] *= inv;
    }
    if (set_scale) {
        double ss = 0;
        for (double v : Zp) ss += v * v;
        const double rms = std::sqrt(ss / std::max<size_t>(Zp.size(), 1));
        s_p_ = rms > 0 ? 1.0 / rms : 1.0;
    }
    for (double &v : Zp) v *= s_p_;
    Z.assign((size_t)n * nf, 0.f);
    for (int s = 0; s < n; ++s) {
        const double th = angles[2 * s], ph = angles[2 * s + 1];
        float *f = Z.data() + (size_t)s * nf;
        for (int m = 1; m <= M; ++m) {
            f[m - 1] = (float)std::cos(m * th);
            f[M + m - 1] = (float)std::sin(m * th);
            f[2 * M + m - 1] = (float)std::cos(m * ph);
            f[3 * M + m - 1] = (float)std::sin(m * ph);
        }
        for (int q = 0; q < np; ++q) f[4 * M + q] = (float)Zp[(size_t)s * np + q];
    }
}

double Mlp::train(int B, const float *X, const float *Y, int epochs, double lr) {
    hipStream_t st = (hipStream_t)stream_;
    int *dstep = nullptr;
    GHIPCHK(hipMalloc(&dstep, sizeof(int)));
    double loss = 0;
    try {
        GHIPCHK(hipMemsetAsync(dstep, 0, sizeof(int), st));
        ensure_batch(B);
        bool graphed = false;
        if (st && epochs > 1) {
            // EPG epochs (forward, backward, Adam with the device-side step
            // count) captured once into a HIP graph and replayed
            constexpr int EPG = 25;
            const int per = std::min(EPG, epochs);
            hipGraph_t g = nullptr;
            GHIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
            try {
                for (int k = 0; k < per; ++k) {
                    loss_grad(B, X, Y, false);
                    adam_scheduled(dstep, lr, epochs);
                }
            } catch (...) {
                hipGraph_t broken = nullptr;
                (void)hipStreamEndCapture(st, &broken);
                if (broken) (void)hipGraphDestroy(broken);
                throw;
            }
            GHIPCHK(hipStreamEndCapture(st, &g));
            hipGraphExec_t ex = nullptr;
            const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            GHIPCHK(e);
            int done = 0;
            for (; done + per <= epochs; done += per) {
                const hipError_t le = hipGraphLaunch(ex, st);
                if (le != hipSuccess) {
                    (void)hipGraphExecDestroy(ex);
                    GHIPCHK(le);
                }
            }
            const hipError_t se = hipStreamSynchronize(st);
            (void)hipGraphExecDestroy(ex);
            GHIPCHK(se);
            for (; done < epochs; ++done) {   // the remainder, launched directly
                loss_grad(B, X, Y, false);
                adam_scheduled(dstep, lr, epochs);
            }
            graphed = true;
        }
        if (!graphed)
            for (int ep = 0; ep < epochs; ++ep) {
                loss_grad(B, X, Y, false);
                adam_scheduled(dstep, lr, epochs);
            }
        loss = loss_grad(B, X, Y, true);
    } catch (...) {
        (void)hipFree(dstep);
        throw;
    }
    (void)hipFree(dstep);
    return loss;
}

double Guess::fit(int n, const double *angles, const void *B, const void *X, const GuessOptions &o) {
    if (n < 1 || n > 512) throw Error(SFMM_E_INVALID_ARG, "learned guess: 1 to 512 training solutions");
    if (o.rank < 1 || o.harmonics < 0 || o.hidden < 1 || o.hidden > 4096 || o.epochs < 0 || !(o.lr > 0) ||
        o.n_theta < 1 || o.n_phi < 1 || (int64_t)o.n_theta * o.n_phi > 4096)
        throw Error(SFMM_E_INVALID_ARG, "learned guess: bad options");
    hipStream_t st = (hipStream_t)stream_;
    o_ = o;
    net_.reset();
    (void)hipFree(W_);
    W_ = nullptr;
    gram_.clear();
    (void)hipFree(Ws_);
    Ws_ = nullptr;
    // POD basis: Gram matrix G[i][j] = <x_i, x_j>, G = V diag(w) V^H,
    // u_k = sum_i x_i V[i][k] / sqrt(w_k) for the r largest w_k
    std::vector<cd> G((size_t)n * n), V;
    std::vector<double> w;
    cross_dots(X, N_, n, X, N_, n, N_, G.data(), stream_);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < i; ++j) {   // symmetrise the rounding
            const cd h = 0.5 * (G[(size_t)i * n + j] + std::conj(G[(size_t)j * n + i]));
            G[(size_t)i * n + j] = h;
            G[(size_t)j * n + i] = std::conj(h);
        }
    hermitian_eig(n, G, w, V);
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](int a, int b) { return w[a] > w[b]; });
    const double wmax = std::max(w[order[0]], 0.0);
    if (!(wmax > 0)) throw Error(SFMM_E_INVALID_ARG, "learned guess: training solutions are all zero");
    int r = std::min(o.rank, n);
    // directions below sqrt(eps) of the largest singular value are not
    // resolved by the Gram matrix
    while (r > 1 && w[order[r - 1]] <= 1e-14 * wmax) --r;
    r_ = r;
    std::vector<cd> coef((size_t)r * n);
    for (int k = 0; k < r; ++k) {
        const double sig = std::sqrt(w[order[k]]);
        for (int i = 0; i < n; ++i) coef[(size_t)k * n + i] = V[(size_t)i * n + order[k]] / sig;
    }
    (void)hipFree(U_);
    U_ = nullptr;
    GHIPCHK(hipMalloc(&U_, sizeof(double2) * (size_t)r * N_));
    lincomb(X, N_, n, coef.data(), r, N_, U_, N_, stream_);
    // features and targets y = s_y Re/Im(U^H x) / ||b||
    std::vector<float> Z;
    std::vector<double> Zp, nb;
    features(n, angles, B, Z, Zp, nb, true);
    const int np = 4 * o.n_theta * o.n_phi, no = 2 * r, nf = 4 * o.harmonics + np;
    std::vector<cd> c((size_t)r * n);
    cross_dots(U_, N_, r, X, N_, n, N_, c.data(), stream_);
    std::vector<double> Y((size_t)n * no);
    for (int s = 0; s < n; ++s) {
        const double inv = nb[s] > 0 ? 1.0 / nb[s] : 0.0;
        for (int k = 0; k < r; ++k) {
            Y[(size_t)s * no + k] = c[(size_t)k * n + s].real() * inv;
            Y[(size_t)s * no + r + k] = c[(size_t)k * n + s].imag() * inv;
        }
    }
    double ss = 0;
    for (double v : Y) ss += v * v;
    const double yrms = std::sqrt(ss / Y.size());
    s_y_ = yrms > 0 ? 1.0 / yrms : 1.0;
    for (double &v : Y) v *= s_y_;
    // linear path (FP64): Ws = Zp^T Gp^+ Y, Gp = Zp Zp^T with eigenvalues at
    // or below 1e-12 of the largest dropped (minimum-norm least squares)
    DevBuf<double> dZp(Zp.size()), dGp((size_t)n * n), dA((size_t)n * no), dLin((size_t)n * no);
    GHIPCHK(hipMemcpyAsync(dZp.p, Zp.data(), sizeof(double) * Zp.size(), hipMemcpyHostToDevice, st));
    dgemm(st, n, n, np, dZp.p, np, 1, dZp.p, 1, np, dGp.p, n);
    std::vector<double> Gp((size_t)n * n);
    GHIPCHK(hipMemcpyAsync(Gp.data(), dGp.p, sizeof(double) * Gp.size(), hipMemcpyDeviceToHost, st));
    GHIPCHK(hipStreamSynchronize(st));
    std::vector<cd> Gc((size_t)n * n), Vg;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Gc[(size_t)i * n + j] = 0.5 * (Gp[(size_t)i * n + j] + Gp[(size_t)j * n + i]);
    std::vector<double> wg;
    hermitian_eig(n, Gc, wg, Vg);
    const double gmax = *std::max_element(wg.begin(), wg.end());
    std::vector<double> A((size_t)n * no, 0.0);   // Gp^+ Y
    for (int k = 0; k < n; ++k) {
        if (!(gmax > 0) || wg[k] <= 1e-12 * gmax) continue;
        for (int q = 0; q < no; ++q) {
            double t = 0;
            for (int i = 0; i < n; ++i) t += Vg[(size_t)i * n + k].real() * Y[(size_t)i * no + q];
            t /= wg[k];
            for (int i = 0; i < n; ++i) A[(size_t)i * no + q] += Vg[(size_t)i * n + k].real() * t;
        }
    }
    GHIPCHK(hipMalloc(&Ws_, sizeof(double) * (size_t)np * no));
    GHIPCHK(hipMemcpyAsync(dA.p, A.data(), sizeof(double) * A.size(), hipMemcpyHostToDevice, st));
    dgemm(st, np, no, n, dZp.p, 1, np, dA.p, no, 1, Ws_, no);
    dgemm(st, n, no, np, dZp.p, np, 1, Ws_, no, 1, dLin.p, no);
    std::vector<double> lin((size_t)n * no);
    GHIPCHK(hipMemcpyAsync(lin.data(), dLin.p, sizeof(double) * lin.size(), hipMemcpyDeviceToHost, st));
    GHIPCHK(hipStreamSynchronize(st));
    // the MLP learns the remainder R = Y - Zp Ws at unit RMS
    ss = 0;
    for (size_t q = 0; q < Y.size(); ++q) ss += (Y[q] - lin[q]) * (Y[q] - lin[q]);
    const double rrms = std::sqrt(ss / Y.size());
    s_r_ = rrms > 0 ? 1.0 / rrms : 1.0;
    std::vector<float> Rs(Y.size());
    for (size_t q = 0; q < Y.size(); ++q) Rs[q] = (float)((Y[q] - lin[q]) * s_r_);
    auto net = std::make_unique<Mlp>(std::vector<int>{nf, o.hidden, o.hidden, no}, stream_);
    net->init_uniform(o.seed, true);
    DevBuf<float> dZ(Z.size()), dR(Rs.size());
    GHIPCHK(hipMemcpyAsync(dZ.p, Z.data(), sizeof(float) * Z.size(), hipMemcpyHostToDevice, st));
    GHIPCHK(hipMemcpyAsync(dR.p, Rs.data(), sizeof(float) * Rs.size(), hipMemcpyHostToDevice, st));
    const double loss = net->train(n, dZ.p, dR.p, o.epochs, o.lr);
    net_ = std::move(net);
    return loss;
}

void Guess::predict(int n, const double *angles, const void *B, void *X0) {
    if (!net_) throw Error(SFMM_E_INVALID_ARG, "learned guess is not trained (call sfmm_guess_fit first)");
    if (n < 1) throw Error(SFMM_E_INVALID_ARG, "n must be positive");
    hipStream_t st = (hipStream_t)stream_;
    std::vector<float> Z;
    std::vector<double> Zp, nb;
    features(n, angles, B, Z, Zp, nb, false);
    const int r = r_, no = 2 * r, np = 4 * o_.n_theta * o_.n_phi;
    DevBuf<float> dZ(Z.size());
    DevBuf<double> dZp(Zp.size()), dLin((size_t)n * no);
    std::vector<float> out((size_t)n * no);
    std::vector<double> lin((size_t)n * no);
    GHIPCHK(hipMemcpyAsync(dZ.p, Z.data(), sizeof(float) * Z.size(), hipMemcpyHostToDevice, st));
    GHIPCHK(hipMemcpyAsync(dZp.p, Zp.data(), sizeof(double) * Zp.size(), hipMemcpyHostToDevice, st));
    dgemm(st, n, no, np, dZp.p, np, 1, Ws_, no, 1, dLin.p, no);
    const float *y = net_->forward(n, dZ.p);
    GHIPCHK(hipMemcpyAsync(out.data(), y, sizeof(float) * out.size(), hipMemcpyDeviceToHost, st));
    GHIPCHK(hipMemcpyAsync(lin.data(), dLin.p, sizeof(double) * lin.size(), hipMemcpyDeviceToHost, st));
    GHIPCHK(hipStreamSynchronize(st));
    std::vector<cd> coef((size_t)n * r);
    for (int s = 0; s < n; ++s)
        for (int k = 0; k < r; ++k) {
            const size_t a = (size_t)s * no + k, b = a + r;
            const double re = (lin[a] + out[a] / s_r_) / s_y_;
            const double im = (lin[b] + out[b] / s_r_) / s_y_;
            coef[(size_t)s * r + k] = cd(re, im) * nb[s];
        }
    lincomb(U_, N_, r, coef.data(), n, N_, X0, N_, stream_);
}

}  // namespace sfmm
