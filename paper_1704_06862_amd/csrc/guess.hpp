// Learned initial guess: device network with hand-written kernels, POD helpers.
#pragma once

#include <cstdint>
#include <functional>
#include <memory>
#include <vector>

#include "core.hpp"

namespace sfmm {

int64_t mlp_param_count(const std::vector<int> &sizes);

// make `device` current for the calling thread
void use_device(int device);

// Multilayer perceptron with tanh hidden layers and a linear output layer.
// Parameters: for every layer W [in][out] row-major, then b [out] (FP32).
class Mlp {
  public:
    Mlp(const std::vector<int> &sizes, void *stream);
    ~Mlp();
    Mlp(const Mlp &) = delete;
    Mlp &operator=(const Mlp &) = delete;
    int64_t n_params() const { return np_; }
    const std::vector<int> &sizes() const { return sizes_; }
    void set_stream(void *s) { stream_ = s; }
    void init_uniform(uint64_t seed, bool zero_last = false);
    void set_params(const float *host);
    void get_params(float *host) const;
    void get_grads(float *host) const;
    // X: device [B][in]; returns device pointer to the [B][out] output
    const float *forward(int B, const float *X);
    // 0.5/B sum ||f(X) - Y||^2 and the gradients (kept on the device); with
    // want_loss = false the loss is not read back (no host synchronisation)
    // and NaN is returned
    double loss_grad(int B, const float *X, const float *Y, bool want_loss = true);
    void adam_step(double lr, double b1 = 0.9, double b2 = 0.999, double eps = 1e-8);
    // Adam step with the step count *step on the device (incremented after
    // the update) and the cosine schedule lr0 (1 + cos(pi (t-1)/epochs)) / 2;
    // launches only kernels, so it can be captured into a graph
    void adam_scheduled(const int *step, double lr0, int epochs, double b1 = 0.9, double b2 = 0.999,
                        double eps = 1e-8);
    // activation buffers for batches up to B (allocates; call before capture)
    void ensure_batch(int B);
    // Adam steps (full batch X [B][in], targets Y [B][out], device), one
    // graph-captured block of steps replayed; returns the final loss
    double train(int B, const float *X, const float *Y, int epochs, double lr);

  private:
    std::vector<int> sizes_;
    void *stream_;
    int64_t np_ = 0;
    float *p_ = nullptr, *g_ = nullptr, *m_ = nullptr, *v_ = nullptr;
    std::vector<float *> acts_;
    float *delta_ = nullptr, *delta2_ = nullptr;
    double *partial_ = nullptr;
    int cap_ = 0;
    int t_ = 0;
};

// Eigen-decomposition of a Hermitian n x n matrix (row-major, overwritten);
// eigenvalues w (unsorted) and eigenvectors as the columns of V.
void hermitian_eig(int n, std::vector<cd> &A, std::vector<double> &w, std::vector<cd> &V);

// out[i][j] = <a_i, b_j> = sum conj(a_i) b_j  (FP64 device vectors of length N)
void cross_dots(const void *A, int64_t lda, int na, const void *B, int64_t ldb, int nbv, int N, cd *out_host,
                void *stream);
// out[i] = ||a_i||
void self_norms(const void *A, int64_t lda, int n, int N, double *out_host, void *stream);
// out_s = sum_j coef[s][j] v_j   (FP64 device vectors of length N)
void lincomb(const void *vecs, int64_t ld, int nv, const cd *coef_host, int ns, int N, void *out, int64_t ldo,
             void *stream);

struct GuessOptions {
    int rank = 72;        // POD basis size r (clamped to the training count)
    int harmonics = 4;    // M angle harmonics
    int hidden = 768;     // width of both tanh hidden layers
    int epochs = 300;     // full-batch Adam steps of the MLP
    double lr = 1e-3;     // peak Adam step, cosine decay to zero
    uint64_t seed = 0;    // weight initialisation
    int n_theta = 16;     // pattern feature grid: theta bands
    int n_phi = 31;       //                       phi samples
};

// b (device, [n][N] complex FP64, boundary layout) read as surface currents:
// F [n][n_dirs][4] (device, FP64) = Re/Im of theta.F, Re/Im of phi.F of its
// far field at dirs [n_dirs][2] (device, theta/phi)
using PatternFn = std::function<void(int n, const void *b, int n_dirs, const double *dirs, double *F)>;

// Learned GMRES initial guess for one body (boundary unknown order).
class Guess {
  public:
    Guess(int N, void *stream, PatternFn pattern) : N_(N), stream_(stream), pattern_(std::move(pattern)) {}
    ~Guess();
    Guess(const Guess &) = delete;
    Guess &operator=(const Guess &) = delete;
    void set_stream(void *s);
    bool trained() const { return net_ != nullptr; }
    int rank() const { return r_; }
    // angles [n][2]; B, X device [n][N] complex (right-hand sides and their
    // solutions).  Returns the final training loss of the MLP (on the
    // unit-RMS remainder of the linear path).
    double fit(int n, const double *angles, const void *B, const void *X, const GuessOptions &o);
    // X0 device [n][N] complex
    void predict(int n, const double *angles, const void *B, void *X0);
    // Baseline without the network: the minimal-residual guess in span(U),
    // c = argmin ||b - Z U c|| (normal equations of W = Z U, W formed once
    // with `product`, which applies Z to r boundary-layout device vectors)
    void span_predict(int n, const void *B, void *X0,
                      const std::function<void(int, const void *, void *)> &product);

  private:
    // features of n right-hand sides: Z [n][nf] (FP32, network input), Zp
    // [n][np] (FP64, the pattern part), ||b||; with `set_scale` the pattern
    // scale s_p is taken from these rows
    void features(int n, const double *angles, const void *B, std::vector<float> &Z, std::vector<double> &Zp,
                  std::vector<double> &nb, bool set_scale);
    int N_;
    void *stream_;
    PatternFn pattern_;
    GuessOptions o_{};
    int r_ = 0;
    void *U_ = nullptr;            // [r][N] complex FP64, orthonormal rows
    double s_p_ = 1, s_y_ = 1, s_r_ = 1;
    double *Ws_ = nullptr;         // [np][2r] FP64 linear path
    std::unique_ptr<Mlp> net_;
    void *W_ = nullptr;            // Z U, [r][N], formed on the first span_predict
    std::vector<cd> gram_;         // W^H W
};

}  // namespace sfmm
