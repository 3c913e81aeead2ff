// Learned initial guess for GMRES (an addition to the paper's method): a
// small MLP trained on the device, with hand-written kernels, on currents the
// solver produced for other incidence angles.
//
//   POD basis   U = first r left singular vectors of X = [x_1 .. x_n]
//               (Gram matrix X^H X on the device, Hermitian Jacobi
//               eigen-decomposition on the host, U = X V Sigma^-1)
//   features    [cos m theta, sin m theta, cos m phi, sin m phi]_{m=1..M},
//               Re/Im (U^H b) / ||b||
//   network     two tanh hidden layers, linear output of Re/Im of the POD
//               coefficients / ||b||; mean-squared error; Adam
//   arithmetic  GEMM operands rounded to bfloat16, products and sums in FP32
//               (exact bf16 x bf16 products, FP32 accumulation), FP32 master
//               weights and optimizer state
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

constexpr int GT = 16;   // GEMM tile

// round-to-nearest-even to bfloat16, returned as float
__device__ __forceinline__ float bf16r(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return __uint_as_float(u & 0xffff0000u);
}

// C[i][j] (=|+=) act( sum_k bf(A(i,k)) bf(B(k,j)) + bias[j] ),
// A(i,k) = A[i*a0 + k*a1], B(k,j) = B[k*b0 + j*b1], C row-major with ldc.
__global__ void __launch_bounds__(GT *GT) k_gemm(int M, int N, int K, const float *__restrict__ A, int64_t a0,
                                                 int64_t a1, const float *__restrict__ B, int64_t b0, int64_t b1,
                                                 const float *__restrict__ bias, int act, float *__restrict__ C,
                                                 int64_t ldc) {
    __shared__ float As[GT][GT + 1], Bs[GT][GT + 1];
    const int ti = threadIdx.x / GT, tj = threadIdx.x % GT;
    const int i = blockIdx.y * GT + ti, j = blockIdx.x * GT + tj;
    float acc = 0.f;
    for (int k0 = 0; k0 < K; k0 += GT) {
        const int ka = k0 + tj, kb = k0 + ti;
        As[ti][tj] = (i < M && ka < K) ? bf16r(A[i * a0 + ka * a1]) : 0.f;
        Bs[ti][tj] = (kb < K && j < N) ? bf16r(B[kb * b0 + j * b1]) : 0.f;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < GT; ++k) acc += As[ti][k] * Bs[k][tj];
        __syncthreads();
    }
    if (i < M && j < N) {
        if (bias) acc += bias[j];
        if (act == 1) acc = tanhf(acc);
        C[i * ldc + j] = acc;
    }
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
    dim3 grid(nb(N, GT), nb(M, GT));
    k_gemm<<<grid, GT * GT, 0, s>>>(M, N, K, A, a0, a1, B, b0, b1, bias, act, C, ldc);
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

void Mlp::init_uniform(uint64_t seed) {
    // SplitMix64 (Steele, Lea, Flood 2014) -> uniform [0,1); weights
    // U(-sqrt(6/(in+out)), +sqrt(6/(in+out))), biases zero
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
        for (int64_t q = 0; q < (int64_t)a * b; ++q) h[off + q] = (float)((2.0 * next() - 1.0) * lim);
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

void Guess::features(int n, const double *angles, const void *B, std::vector<float> &F, std::vector<double> &nb) {
    const int M = o_.harmonics, r = r_, nf = 4 * M + 2 * r;
    nb.assign(n, 0.0);
    self_norms(B, N_, n, N_, nb.data(), stream_);
    std::vector<cd> proj((size_t)r * n);
    cross_dots(U_, N_, r, B, N_, n, N_, proj.data(), stream_);   // proj[k][s] = u_k^H b_s
    F.assign((size_t)n * nf, 0.f);
    for (int s = 0; s < n; ++s) {
        const double th = angles[2 * s], ph = angles[2 * s + 1];
        float *f = F.data() + (size_t)s * nf;
        for (int m = 1; m <= M; ++m) {
            f[m - 1] = (float)std::cos(m * th);
            f[M + m - 1] = (float)std::sin(m * th);
            f[2 * M + m - 1] = (float)std::cos(m * ph);
            f[3 * M + m - 1] = (float)std::sin(m * ph);
        }
        const double inv = nb[s] > 0 ? 1.0 / nb[s] : 0.0;
        for (int k = 0; k < r; ++k) {
            const cd p = proj[(size_t)k * n + s] * inv;
            f[4 * M + k] = (float)p.real();
            f[4 * M + r + k] = (float)p.imag();
        }
    }
}

double Guess::fit(int n, const double *angles, const void *B, const void *X, const GuessOptions &o) {
    if (n < 1 || n > 512) throw Error(SFMM_E_INVALID_ARG, "learned guess: 1 to 512 training solutions");
    if (o.rank < 1 || o.harmonics < 0 || o.hidden < 1 || o.epochs < 0 || !(o.lr > 0))
        throw Error(SFMM_E_INVALID_ARG, "learned guess: bad options");
    o_ = o;
    net_.reset();
    (void)hipFree(W_);
    W_ = nullptr;
    gram_.clear();
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
    // features and standardised targets Re/Im(U^H x) / ||b||
    std::vector<float> F;
    std::vector<double> nb;
    features(n, angles, B, F, nb);
    std::vector<cd> c((size_t)r * n);
    cross_dots(U_, N_, r, X, N_, n, N_, c.data(), stream_);
    const int no = 2 * r, nf = 4 * o.harmonics + 2 * r;
    std::vector<double> Yd((size_t)n * no);
    for (int s = 0; s < n; ++s) {
        const double inv = nb[s] > 0 ? 1.0 / nb[s] : 0.0;
        for (int k = 0; k < r; ++k) {
            Yd[(size_t)s * no + k] = c[(size_t)k * n + s].real() * inv;
            Yd[(size_t)s * no + r + k] = c[(size_t)k * n + s].imag() * inv;
        }
    }
    mu_.assign(no, 0.0);
    sd_.assign(no, 0.0);
    for (int j = 0; j < no; ++j) {
        for (int s = 0; s < n; ++s) mu_[j] += Yd[(size_t)s * no + j];
        mu_[j] /= n;
        for (int s = 0; s < n; ++s) sd_[j] += (Yd[(size_t)s * no + j] - mu_[j]) * (Yd[(size_t)s * no + j] - mu_[j]);
        sd_[j] = std::sqrt(sd_[j] / n);
    }
    const double sdmax = *std::max_element(sd_.begin(), sd_.end());
    for (double &v : sd_) v = std::max(v, sdmax > 0 ? 1e-6 * sdmax : 1.0);
    std::vector<float> Y((size_t)n * no);
    for (int s = 0; s < n; ++s)
        for (int j = 0; j < no; ++j) Y[(size_t)s * no + j] = (float)((Yd[(size_t)s * no + j] - mu_[j]) / sd_[j]);
    // train on the device: full batch, Adam, cosine step decay
    auto net = std::make_unique<Mlp>(std::vector<int>{nf, o.hidden, o.hidden, no}, stream_);
    net->init_uniform(o.seed);
    float *dF = nullptr, *dY = nullptr;
    int *dstep = nullptr;
    GHIPCHK(hipMalloc(&dF, sizeof(float) * F.size()));
    GHIPCHK(hipMalloc(&dY, sizeof(float) * Y.size()));
    GHIPCHK(hipMalloc(&dstep, sizeof(int)));
    double loss = 0;
    try {
        GHIPCHK(hipMemcpyAsync(dF, F.data(), sizeof(float) * F.size(), hipMemcpyHostToDevice, (hipStream_t)stream_));
        GHIPCHK(hipMemcpyAsync(dY, Y.data(), sizeof(float) * Y.size(), hipMemcpyHostToDevice, (hipStream_t)stream_));
        // one epoch (forward, backward, Adam with the device-side step count)
        // is captured once into a HIP graph and replayed
        GHIPCHK(hipMemsetAsync(dstep, 0, sizeof(int), (hipStream_t)stream_));
        net->ensure_batch(n);
        hipStream_t st = (hipStream_t)stream_;
        bool graphed = false;
        if (st && o.epochs > 1) {
            hipGraph_t g = nullptr;
            // EPG epochs per graph launch
            constexpr int EPG = 25;
            const int per = std::min(EPG, o.epochs);
            GHIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
            try {
                for (int k = 0; k < per; ++k) {
                    net->loss_grad(n, dF, dY, false);
                    net->adam_scheduled(dstep, o.lr, o.epochs);
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
            for (; done + per <= o.epochs; done += per) {
                const hipError_t le = hipGraphLaunch(ex, st);
                if (le != hipSuccess) {
                    (void)hipGraphExecDestroy(ex);
                    GHIPCHK(le);
                }
            }
            GHIPCHK(hipStreamSynchronize(st));
            (void)hipGraphExecDestroy(ex);
            for (; done < o.epochs; ++done) {   // the remainder, launched directly
                net->loss_grad(n, dF, dY, false);
                net->adam_scheduled(dstep, o.lr, o.epochs);
            }
            graphed = true;
        }
        if (!graphed)
            for (int ep = 0; ep < o.epochs; ++ep) {
                net->loss_grad(n, dF, dY, false);
                net->adam_scheduled(dstep, o.lr, o.epochs);
            }
        loss = net->loss_grad(n, dF, dY, true);
    } catch (...) {
        (void)hipFree(dF);
        (void)hipFree(dY);
        (void)hipFree(dstep);
        throw;
    }
    (void)hipFree(dF);
    (void)hipFree(dY);
    (void)hipFree(dstep);
    net_ = std::move(net);
    return loss;
}

void Guess::predict(int n, const double *angles, const void *B, void *X0) {
    if (!net_) throw Error(SFMM_E_INVALID_ARG, "learned guess is not trained (call sfmm_guess_fit first)");
    if (n < 1) throw Error(SFMM_E_INVALID_ARG, "n must be positive");
    std::vector<float> F;
    std::vector<double> nb;
    features(n, angles, B, F, nb);
    const int r = r_, no = 2 * r, nf = 4 * o_.harmonics + 2 * r;
    float *dF = nullptr;
    GHIPCHK(hipMalloc(&dF, sizeof(float) * F.size()));
    std::vector<float> out((size_t)n * no);
    try {
        GHIPCHK(hipMemcpyAsync(dF, F.data(), sizeof(float) * F.size(), hipMemcpyHostToDevice, (hipStream_t)stream_));
        const float *y = net_->forward(n, dF);
        GHIPCHK(hipMemcpyAsync(out.data(), y, sizeof(float) * out.size(), hipMemcpyDeviceToHost,
                               (hipStream_t)stream_));
        GHIPCHK(hipStreamSynchronize((hipStream_t)stream_));
    } catch (...) {
        (void)hipFree(dF);
        throw;
    }
    (void)hipFree(dF);
    (void)nf;
    std::vector<cd> coef((size_t)n * r);
    for (int s = 0; s < n; ++s)
        for (int k = 0; k < r; ++k) {
            const double re = out[(size_t)s * no + k] * sd_[k] + mu_[k];
            const double im = out[(size_t)s * no + r + k] * sd_[r + k] + mu_[r + k];
            coef[(size_t)s * r + k] = cd(re, im) * nb[s];
        }
    lincomb(U_, N_, r, coef.data(), n, N_, X0, N_, stream_);
}

}  // namespace sfmm
