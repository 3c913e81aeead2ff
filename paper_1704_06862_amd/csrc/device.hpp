// Interface between the host core / C ABI and the HIP implementation.
#pragma once

#include <memory>

#include "core.hpp"

namespace sfmm {

// Everything built on the host for one body.
struct BodyHost {
    Mesh mesh;
    Octree oct;
    NearMatrix near;
    IluFactors ilu;
    std::vector<RegionTables> tables;   // parallel to oct.regions
    int precond = SFMM_PRECOND_ILU0;
    int form = SFMM_FORM_PMCHWT;        // integral equation (SFMM_FORM_*)
    std::vector<cd> poly;               // roots of the polynomial preconditioner
    std::vector<cd> poly_dinv;          // its edge-block scaling D^-1, [position][4]
};

struct StageTimes {
    double ms[8] = {0};
    int64_t n[8] = {0};
};

// Device-resident body.  Vectors at this interface are complex FP64 in the
// boundary layout ([n_rhs][2E], J then M~) on the device unless noted.
class DeviceBody {
  public:
    virtual ~DeviceBody() = default;
    virtual void matvec(int n_rhs, const void *x_dev, void *y_dev, int parts) = 0;
    virtual void precond(int n_rhs, const void *x_dev, void *y_dev) = 0;
    // solver: SFMM_SOLVER_* (GMRES(restart), BiCGStab or CGS)
    virtual void solve(int solver, int n_rhs, const void *b_dev, void *x_dev, const void *x0_dev, int restart,
                       int max_iters, double tol, sfmm_solve_info *info, int verbose) = 0;
    virtual void planewave_rhs(int n_rhs, const double *angles_host, const double *pol_host, void *b_dev) = 0;
    virtual void rcs(int n_rhs, const void *x_dev, int n_dirs, const double *theta_phi_host, double *sigma_host) = 0;
    // as rcs, staged through the library's static device scratch instead of
    // allocated buffers (n_dirs * (2 + 2 n_rhs) <= noalloc_scratch_doubles())
    virtual void rcs_noalloc(int n_rhs, const void *x_dev, int n_dirs, const double *theta_phi_host,
                             double *sigma_host) = 0;
    // the far field of x read as surface currents (FP64, on the device):
    // F_dev [n_rhs][n_dirs][4] = Re/Im of theta.F, Re/Im of phi.F at the
    // directions dirs_dev [n_dirs][2] (theta, phi)
    virtual void far_pattern(int n_rhs, const void *x_dev, int n_dirs, const double *dirs_dev, double *F_dev) = 0;
    virtual void set_stream(void *stream) = 0;
    // the stream all of this body's work is ordered on (the context's stream,
    // or a stream of the body's own when the context has none)
    virtual void *stream() const = 0;
    virtual void stream_synchronize() = 0;
    virtual void profile(bool enable) = 0;
    virtual StageTimes times() const = 0;
    virtual int64_t device_bytes() const = 0;
};

std::unique_ptr<DeviceBody> make_device_body(const BodyHost &h, int precision, int device, void *stream,
                                             bool graphs, bool autotune, int kernel_plan, int verbose);

// The near-field matrix of fill_near computed on the device (one thread per
// stored edge pair) and copied back to the host.
NearMatrix fill_near_device(const Mesh &m, const Octree &o, int form, int device);
// factor_ilu on the device (the same block factorisation and folded form).
IluFactors factor_ilu_device(const Octree &o, const NearMatrix &Z, double pivot_tol, int device);

// HIP helpers used by the C ABI for host <-> device staging.
void *device_alloc(size_t bytes);
void device_free(void *p);
void copy_h2d(void *dst, const void *src, size_t bytes, void *stream);
void copy_d2h(void *dst, const void *src, size_t bytes, void *stream);
void stream_sync(void *stream);
void check_device(int device);
size_t noalloc_scratch_doubles();

}  // namespace sfmm
