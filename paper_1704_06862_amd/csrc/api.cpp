// C ABI of the sfmm library (declared in include/sfmm.h).  Argument
// validation, host setup, host <-> device staging and error capture; all
// products, preconditioner solves and Krylov steps run in the HIP kernels.
#include <algorithm>
#include <cmath>
#include <atomic>
#include <chrono>
#include <functional>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <thread>

#include "device.hpp"
#include "guess.hpp"

using namespace sfmm;

struct sfmm_ctx {
    sfmm_options opt{};
    std::vector<std::unique_ptr<BodyHost>> bodies;
    std::vector<std::unique_ptr<DeviceBody>> dev;
    std::vector<std::unique_ptr<Guess>> guess;
    void *stream = nullptr;
    std::string err;
    bool poisoned = false;
};

namespace {

thread_local std::string g_setup_error;

// Rounding amplification of the diagonal translation operator at a level's
// closest offset (two boxes apart, kX = k 2a): the operator is a sum over
// n <= L of (2n + 1) h_n(kX) terms, which grow like y_n(kX) once n > kX,
// while the translated field is of the order of h_0(kX) ~ 1 / kX.  Returns
// kX sum_n (2n + 1) (|y_n(kX)| + 1 / kX), y_n by the upward recurrence
// y_{n+1} = (2n + 1) / z y_n - y_{n-1} (stable for y_n).
double translation_amplification(double kx, int L) {
    double ym = -std::cos(kx) / kx;                               // y_0
    double y = -std::cos(kx) / (kx * kx) - std::sin(kx) / kx;      // y_1
    double b = std::fabs(ym) + 1.0 / kx;
    if (L >= 1) b += 3.0 * (std::fabs(y) + 1.0 / kx);
    for (int n = 1; n < L; ++n) {
        const double yn = (2 * n + 1) / kx * y - ym;
        ym = y;
        y = yn;
        b += (2 * n + 3) * (std::fabs(y) + 1.0 / kx);
    }
    return b * kx;
}

// FP32 storage of the translation tables is refused where single-precision
// rounding (6e-8) times that amplification exceeds 5: measured, an estimate of
// 276 gave a product error of 0.12 and estimates below 0.02 left FP32 products
// at the FP64 accuracy.
void check_fp32_translations(const BodyHost &bh) {
    for (const RegionTree &rt : bh.oct.regions) {
        const double k = std::abs(bh.mesh.k[rt.region]);
        for (size_t l = 2; l < rt.levels_L.size() && l < rt.lev.size(); ++l) {
            if (rt.lev[l].key.empty()) continue;
            const double amp = 6e-8 * translation_amplification(k * 2.0 * rt.lev[l].a, rt.levels_L[l]);
            if (amp > 5.0) {
                char msg[320];
                std::snprintf(msg, sizeof msg,
                              "region %d level %zu: truncation order %d at kX = %.2f amplifies FP32 rounding about "
                              "%.3g-fold; use precision FP64, fewer extra multipoles or larger boxes",
                              rt.region, l, rt.levels_L[l], k * 2.0 * rt.lev[l].a, amp / 6e-8);
                throw Error(SFMM_E_UNSUPPORTED, msg);
            }
        }
    }
}

template <typename F>
sfmm_status guarded(sfmm_ctx *ctx, F &&fn) {
    try {
        if (ctx && ctx->poisoned) throw Error(SFMM_E_DEVICE, "context unusable after an earlier device error");
        fn();
        return SFMM_OK;
    } catch (const Error &e) {
        if (ctx) {
            ctx->err = e.what();
            if (e.code == SFMM_E_DEVICE) ctx->poisoned = true;
        } else {
            g_setup_error = e.what();
        }
        return e.code;
    } catch (const std::bad_alloc &) {
        if (ctx) ctx->err = "host allocation failed";
        else g_setup_error = "host allocation failed";
        return SFMM_E_OOM;
    } catch (const std::exception &e) {
        if (ctx) ctx->err = e.what();
        else g_setup_error = e.what();
        return SFMM_E_INVALID_ARG;
    }
}

const BodyHost &body_of(const sfmm_ctx *ctx, int32_t body) {
    if (!ctx) throw Error(SFMM_E_INVALID_ARG, "NULL context");
    if (body < 0 || body >= (int32_t)ctx->bodies.size()) throw Error(SFMM_E_INVALID_ARG, "body index out of range");
    return *ctx->bodies[body];
}

DeviceBody &dev_of(sfmm_ctx *ctx, int32_t body) {
    body_of(ctx, body);
    if (ctx->dev.empty() || !ctx->dev[body])
        throw Error(SFMM_E_INVALID_ARG, "context was built with device = -1 (host tables only)");
    return *ctx->dev[body];
}

// RAII staging buffer for host pointers
struct Staged {
    void *p = nullptr;
    explicit Staged(size_t bytes) : p(device_alloc(bytes)) {}
    ~Staged() { device_free(p); }
};

void solve_one(sfmm_ctx *ctx, int32_t body, int32_t n_rhs, const void *b, void *x, const void *x0,
               sfmm_solve_info *info, int32_t on_device) {
    DeviceBody &d = dev_of(ctx, body);
    if (n_rhs <= 0 || !b || !x) throw Error(SFMM_E_INVALID_ARG, "bad arguments");
    const sfmm_options &o = ctx->opt;
    const size_t bytes = (size_t)n_rhs * 2 * ctx->bodies[body]->mesh.ne * 2 * sizeof(double);
    if (on_device) {
        d.solve(o.solver, n_rhs, b, x, x0, o.gmres_restart, o.max_iters, o.tol, info, o.verbose);
        return;
    }
    Staged db(bytes), dx(bytes);
    std::unique_ptr<Staged> dx0;
    copy_h2d(db.p, b, bytes, d.stream());
    if (x0) {
        dx0 = std::make_unique<Staged>(bytes);
        copy_h2d(dx0->p, x0, bytes, d.stream());
    }
    try {
        d.solve(o.solver, n_rhs, db.p, dx.p, dx0 ? dx0->p : nullptr, o.gmres_restart, o.max_iters, o.tol, info,
                o.verbose);
    } catch (const Error &e) {
        if (e.code == SFMM_E_NOT_CONVERGED) copy_d2h(x, dx.p, bytes, d.stream());
        throw;
    }
    copy_d2h(x, dx.p, bytes, d.stream());
}

}  // namespace

extern "C" {

void sfmm_default_options(sfmm_options *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->finest_box = 0.0;
    o->n_levels = 0;
    o->digits = 3.0;
    o->extra_multipoles = 0;
    o->precision = SFMM_PREC_FP32;
    o->gmres_restart = 30;
    o->max_iters = 1000;
    o->tol = 1e-6;
    o->device = 0;
    o->verbose = 0;
    o->preconditioner = SFMM_PRECOND_POLY;
    o->poly_degree = 16;
    o->graphs = 1;
    o->autotune = 0;
    o->kernel_plan = 0;
    o->formulation = SFMM_FORM_PMCHWT;
    o->quad_points = 7;
    o->solver = SFMM_SOLVER_GMRES;
    o->ilu_pivot_tol = 1e-13;
    o->setup_on_device = -1;
}

sfmm_status sfmm_setup(const sfmm_body *bodies, int32_t n_bodies, const sfmm_options *opt, sfmm_ctx **out) {
    return guarded(nullptr, [&] {
        if (!out) throw Error(SFMM_E_INVALID_ARG, "out is NULL");
        *out = nullptr;
        if (!bodies || n_bodies <= 0) throw Error(SFMM_E_INVALID_ARG, "no bodies");
        auto ctx = std::make_unique<sfmm_ctx>();
        if (opt) ctx->opt = *opt;
        else sfmm_default_options(&ctx->opt);
        sfmm_options &o = ctx->opt;
        if (o.gmres_restart <= 0) o.gmres_restart = 30;
        if (o.max_iters <= 0) o.max_iters = 1000;
        if (!(o.tol > 0)) o.tol = 1e-6;
        if (o.precision != SFMM_PREC_FP32 && o.precision != SFMM_PREC_FP64 && o.precision != SFMM_PREC_BF16_SPLIT)
            throw Error(SFMM_E_INVALID_ARG, "unknown precision");
        if (o.extra_multipoles < 0 || o.extra_multipoles > 64) throw Error(SFMM_E_INVALID_ARG, "extra_multipoles out of range");
        if (o.preconditioner < 0 || o.preconditioner > 3) throw Error(SFMM_E_INVALID_ARG, "unknown preconditioner");
        if (o.poly_degree <= 0) o.poly_degree = 16;
        if (o.poly_degree > 64) throw Error(SFMM_E_INVALID_ARG, "poly_degree must be at most 64");
        if (o.quad_points == 0) o.quad_points = 7;
        if (o.quad_points != 7) throw Error(SFMM_E_UNSUPPORTED, "only the 7-point triangle rule is built");
        if (o.formulation < SFMM_FORM_PMCHWT || o.formulation > SFMM_FORM_CNF)
            throw Error(SFMM_E_UNSUPPORTED, "unknown formulation");
        if (o.solver < SFMM_SOLVER_GMRES || o.solver > SFMM_SOLVER_CGS) throw Error(SFMM_E_UNSUPPORTED, "unknown solver");
        if (o.ilu_pivot_tol == 0) o.ilu_pivot_tol = 1e-13;
        if (!(o.ilu_pivot_tol > 0) || !std::isfinite(o.ilu_pivot_tol))
            throw Error(SFMM_E_INVALID_ARG, "ilu_pivot_tol must be positive");
        if (!std::isfinite(o.finest_box) || o.finest_box < 0 || !std::isfinite(o.digits) || o.digits < 0)
            throw Error(SFMM_E_INVALID_ARG, "finest_box and digits must be finite and non-negative");
        if (o.setup_on_device < -1 || o.setup_on_device > 1)
            throw Error(SFMM_E_INVALID_ARG, "setup_on_device must be -1, 0 or 1");
        if (o.setup_on_device == 1 && o.device < 0)
            throw Error(SFMM_E_INVALID_ARG, "setup_on_device needs a device");
        if (o.setup_on_device == -1) o.setup_on_device = o.device >= 0 ? 1 : 0;
        if (o.device >= 0) check_device(o.device);
        for (int32_t i = 0; i < n_bodies; ++i) {
            auto t0 = std::chrono::steady_clock::now();
            auto bh = std::make_unique<BodyHost>();
            bh->mesh = build_mesh(bodies[i]);
            bh->oct = build_octree(bh->mesh, o.finest_box, o.n_levels, o.digits, o.extra_multipoles);
            if (o.precision != SFMM_PREC_FP64) check_fp32_translations(*bh);
            auto t1 = std::chrono::steady_clock::now();
            bh->form = o.formulation;
            bh->near = o.setup_on_device ? fill_near_device(bh->mesh, bh->oct, o.formulation, o.device)
                                             : fill_near(bh->mesh, bh->oct, o.formulation);
            auto t2 = std::chrono::steady_clock::now();
            if (o.preconditioner == SFMM_PRECOND_ILU0)
                bh->ilu = o.setup_on_device ? factor_ilu_device(bh->oct, bh->near, o.ilu_pivot_tol, o.device)
                                            : factor_ilu(bh->mesh, bh->oct, bh->near, o.ilu_pivot_tol);
            else if (o.preconditioner == SFMM_PRECOND_BLOCK_JACOBI) bh->ilu = factor_block_jacobi(bh->mesh, bh->oct, bh->near, o.ilu_pivot_tol);
            else if (o.preconditioner == SFMM_PRECOND_POLY) {
                bh->poly_dinv = edge_block_inverse(bh->oct, bh->near);
                bh->poly = poly_roots(bh->mesh, bh->oct, bh->near, o.poly_degree, bh->poly_dinv);
            }
            bh->precond = o.preconditioner;
            auto t3 = std::chrono::steady_clock::now();
            for (const RegionTree &rt : bh->oct.regions) bh->tables.push_back(build_tables(bh->mesh, bh->oct, rt, o.formulation));
            auto t4 = std::chrono::steady_clock::now();
            if (o.verbose) {
                auto s = [](auto a, auto b) { return std::chrono::duration<double>(b - a).count(); };
                std::fprintf(stderr,
                             "sfmm: body %d: %d edges, %d levels, %d finest boxes, %lld near pairs, %lld translation "
                             "pairs; octree %.2fs near %.2fs ilu %.2fs tables %.2fs\n",
                             i, bh->mesh.ne, bh->oct.nlev, bh->oct.nb, (long long)bh->oct.near_pairs,
                             (long long)bh->oct.trans_pairs, s(t0, t1), s(t1, t2), s(t2, t3), s(t3, t4));
            }
            ctx->bodies.push_back(std::move(bh));
        }
        if (o.device >= 0) {
            for (auto &bh : ctx->bodies) ctx->dev.push_back(make_device_body(*bh, o.precision, o.device, ctx->stream, o.graphs != 0,
                                                                         o.autotune != 0, o.kernel_plan, o.verbose));
        }
        *out = ctx.release();
    });
}

void sfmm_destroy(sfmm_ctx *ctx) {
    if (!ctx) return;
    try {
        ctx->guess.clear();
        ctx->dev.clear();
    } catch (...) {
    }
    delete ctx;
}

const char *sfmm_last_error(const sfmm_ctx *ctx) { return ctx ? ctx->err.c_str() : g_setup_error.c_str(); }

sfmm_status sfmm_set_stream(sfmm_ctx *ctx, void *stream) {
    return guarded(ctx, [&] {
        if (!ctx) throw Error(SFMM_E_INVALID_ARG, "NULL context");
        ctx->stream = stream;
        for (auto &d : ctx->dev)
            if (d) d->set_stream(stream);
        for (size_t b = 0; b < ctx->guess.size() && b < ctx->dev.size(); ++b)
            if (ctx->guess[b] && ctx->dev[b]) ctx->guess[b]->set_stream(ctx->dev[b]->stream());
    });
}

sfmm_status sfmm_set_solver(sfmm_ctx *ctx, int32_t gmres_restart, int32_t max_iters, double tol) {
    return guarded(ctx, [&] {
        if (!ctx) throw Error(SFMM_E_INVALID_ARG, "NULL context");
        if (gmres_restart < 0 || gmres_restart > 1000 || max_iters < 0 || !(tol >= 0))
            throw Error(SFMM_E_INVALID_ARG, "bad solver settings");
        if (gmres_restart > 0) ctx->opt.gmres_restart = gmres_restart;
        if (max_iters > 0) ctx->opt.max_iters = max_iters;
        if (tol > 0) ctx->opt.tol = tol;
    });
}

sfmm_status sfmm_set_krylov(sfmm_ctx *ctx, int32_t solver) {
    return guarded(ctx, [&] {
        if (!ctx) throw Error(SFMM_E_INVALID_ARG, "NULL context");
        if (solver < SFMM_SOLVER_GMRES || solver > SFMM_SOLVER_CGS) throw Error(SFMM_E_INVALID_ARG, "unknown solver");
        ctx->opt.solver = solver;
    });
}

sfmm_status sfmm_num_unknowns(const sfmm_ctx *ctx, int32_t body, int64_t *n) {
    return guarded(const_cast<sfmm_ctx *>(ctx), [&] {
        const BodyHost &b = body_of(ctx, body);
        if (!n) throw Error(SFMM_E_INVALID_ARG, "NULL output");
        *n = 2 * (int64_t)b.mesh.ne;
    });
}

sfmm_status sfmm_edges(const sfmm_ctx *ctx, int32_t body, int32_t *ev) {
    return guarded(const_cast<sfmm_ctx *>(ctx), [&] {
        const BodyHost &b = body_of(ctx, body);
        if (!ev) throw Error(SFMM_E_INVALID_ARG, "NULL output");
        for (int e = 0; e < b.mesh.ne; ++e) {
            ev[2 * e] = b.mesh.ev[e][0];
            ev[2 * e + 1] = b.mesh.ev[e][1];
        }
    });
}

static void vector_call(sfmm_ctx *ctx, int32_t body, int32_t n_rhs, const void *x, void *y, int32_t on_device,
                        const std::function<void(DeviceBody &, const void *, void *)> &fn) {
    DeviceBody &d = dev_of(ctx, body);
    if (n_rhs <= 0 || !x || !y) throw Error(SFMM_E_INVALID_ARG, "bad vector arguments");
    const size_t bytes = (size_t)n_rhs * 2 * ctx->bodies[body]->mesh.ne * 2 * sizeof(double);
    if (on_device) {
        fn(d, x, y);
    } else {
        Staged dx(bytes), dy(bytes);
        copy_h2d(dx.p, x, bytes, d.stream());
        fn(d, dx.p, dy.p);
        copy_d2h(y, dy.p, bytes, d.stream());
    }
}

sfmm_status sfmm_matvec(sfmm_ctx *ctx, int32_t body, int32_t n_rhs, const void *x, void *y, int32_t on_device,
                        int32_t parts) {
    return guarded(ctx, [&] {
        if (parts < 1 || parts > 3) throw Error(SFMM_E_INVALID_ARG, "parts must be 1, 2 or 3");
        vector_call(ctx, body, n_rhs, x, y, on_device,
                    [&](DeviceBody &d, const void *a, void *b) { d.matvec(n_rhs, a, b, parts); });
    });
}

sfmm_status sfmm_precond(sfmm_ctx *ctx, int32_t body, int32_t n_rhs, const void *x, void *y, int32_t on_device) {
    return guarded(ctx, [&] {
        vector_call(ctx, body, n_rhs, x, y, on_device,
                    [&](DeviceBody &d, const void *a, void *b) { d.precond(n_rhs, a, b); });
    });
}

sfmm_status sfmm_planewave_rhs(sfmm_ctx *ctx, int32_t body, int32_t n_rhs, const double *angles, const double *pol,
                               void *b, int32_t on_device) {
    return guarded(ctx, [&] {
        DeviceBody &d = dev_of(ctx, body);
        if (n_rhs <= 0 || !angles || !b) throw Error(SFMM_E_INVALID_ARG, "bad arguments");
        const size_t bytes = (size_t)n_rhs * 2 * ctx->bodies[body]->mesh.ne * 2 * sizeof(double);
        if (on_device) {
            d.planewave_rhs(n_rhs, angles, pol, b);
        } else {
            Staged db(bytes);
            d.planewave_rhs(n_rhs, angles, pol, db.p);
            copy_d2h(b, db.p, bytes, d.stream());
        }
    });
}

sfmm_status sfmm_solve(sfmm_ctx *ctx, int32_t body, int32_t n_rhs, const void *b, void *x, const void *x0,
                       sfmm_solve_info *info, int32_t on_device) {
    return guarded(ctx, [&] { solve_one(ctx, body, n_rhs, b, x, x0, info, on_device); });
}

sfmm_status sfmm_solve_bodies(sfmm_ctx *ctx, int32_t n, const int32_t *bodies, const int32_t *n_rhs,
                              const void *const *b, void *const *x, sfmm_solve_info *info, int32_t on_device) {
    return guarded(ctx, [&] {
        if (!ctx || n <= 0 || !bodies || !n_rhs || !b || !x) throw Error(SFMM_E_INVALID_ARG, "bad arguments");
        std::vector<int64_t> off(n + 1, 0);
        std::vector<char> seen(ctx->bodies.size(), 0);
        for (int i = 0; i < n; ++i) {
            dev_of(ctx, bodies[i]);
            if (n_rhs[i] <= 0 || !b[i] || !x[i]) throw Error(SFMM_E_INVALID_ARG, "bad arguments for one body");
            if (seen[bodies[i]]) throw Error(SFMM_E_INVALID_ARG, "a body is listed twice");
            seen[bodies[i]] = 1;
            off[i + 1] = off[i] + n_rhs[i];
        }
        // largest work first, so uneven bodies finish close together
        std::vector<int> order(n);
        for (int i = 0; i < n; ++i) order[i] = i;
        std::sort(order.begin(), order.end(), [&](int a, int c) {
            return (int64_t)ctx->bodies[bodies[a]]->mesh.ne * n_rhs[a] > (int64_t)ctx->bodies[bodies[c]]->mesh.ne * n_rhs[c];
        });
        if (ctx->stream) stream_sync(ctx->stream);   // inputs made on the context stream are complete
        std::vector<sfmm_status> codes(n, SFMM_OK);
        std::vector<std::string> msgs(n);
        std::atomic<int> next{0};
        auto worker = [&] {
            try {
                use_device(ctx->opt.device);
            } catch (const Error &e) {
                next = n;
                codes[0] = e.code;
                msgs[0] = e.what();
                return;
            }
            for (;;) {
                const int k = next++;
                if (k >= n) break;
                const int i = order[k];
                DeviceBody &d = *ctx->dev[bodies[i]];
                // each body runs on a stream of its own while this call lasts
                d.set_stream(nullptr);
                try {
                    solve_one(ctx, bodies[i], n_rhs[i], b[i], x[i], nullptr, info ? info + off[i] : nullptr,
                              on_device);
                    d.stream_synchronize();
                } catch (const Error &e) {
                    codes[i] = e.code;
                    msgs[i] = e.what();
                } catch (const std::exception &e) {
                    codes[i] = SFMM_E_INVALID_ARG;
                    msgs[i] = e.what();
                }
                d.set_stream(ctx->stream);
            }
        };
        const int nw = std::min(n, 8);
        std::vector<std::thread> pool;
        for (int w = 0; w < nw; ++w) pool.emplace_back(worker);
        for (std::thread &t : pool) t.join();
        int worst = -1;
        for (int i = 0; i < n; ++i) {
            if (codes[i] == SFMM_OK) continue;
            if (worst < 0 || (codes[worst] == SFMM_E_NOT_CONVERGED && codes[i] != SFMM_E_NOT_CONVERGED)) worst = i;
        }
        if (worst >= 0) throw Error(codes[worst], "body " + std::to_string(bodies[worst]) + ": " + msgs[worst]);
    });
}

sfmm_status sfmm_rcs(sfmm_ctx *ctx, int32_t body, int32_t n_rhs, const void *x, int32_t n_dirs,
                     const double *theta_phi, double *sigma, int32_t on_device) {
    return guarded(ctx, [&] {
        DeviceBody &d = dev_of(ctx, body);
        if (n_rhs <= 0 || n_dirs <= 0 || !x || !theta_phi || !sigma) throw Error(SFMM_E_INVALID_ARG, "bad arguments");
        const size_t bytes = (size_t)n_rhs * 2 * ctx->bodies[body]->mesh.ne * 2 * sizeof(double);
        if (on_device) {
            d.rcs(n_rhs, x, n_dirs, theta_phi, sigma);
        } else {
            Staged dx(bytes);
            copy_h2d(dx.p, x, bytes, d.stream());
            d.rcs(n_rhs, dx.p, n_dirs, theta_phi, sigma);
        }
    });
}

sfmm_status sfmm_rcs_noalloc(sfmm_ctx *ctx, int32_t body, int32_t n_rhs, const void *x_dev, int32_t n_dirs,
                             const double *theta_phi, double *sigma) {
    return guarded(ctx, [&] {
        DeviceBody &d = dev_of(ctx, body);
        if (n_rhs <= 0 || n_dirs <= 0 || !x_dev || !theta_phi || !sigma)
            throw Error(SFMM_E_INVALID_ARG, "bad arguments");
        d.rcs_noalloc(n_rhs, x_dev, n_dirs, theta_phi, sigma);
    });
}

sfmm_status sfmm_near_rows(const sfmm_ctx *ctx, int32_t body, int32_t n_rows, const int32_t *edges, double *out) {
    return guarded(const_cast<sfmm_ctx *>(ctx), [&] {
        const BodyHost &b = body_of(ctx, body);
        if (n_rows <= 0 || !edges || !out) throw Error(SFMM_E_INVALID_ARG, "bad arguments");
        const int ne = b.mesh.ne;
        const Octree &o = b.oct;
        const size_t row_len = (size_t)2 * ne * 2;  // doubles per row
        std::memset(out, 0, sizeof(double) * row_len * 2 * n_rows);
        // box of every internal position
        std::vector<int> box_of(ne);
        for (int bx = 0; bx < o.nb; ++bx)
            for (int p = o.bstart[bx]; p < o.bstart[bx + 1]; ++p) box_of[p] = bx;
        for (int i = 0; i < n_rows; ++i) {
            int e = edges[i];
            if (e < 0 || e >= ne) throw Error(SFMM_E_INVALID_ARG, "edge index out of range");
            int p = o.pos[e];
            int bx = box_of[p];
            int row = p - o.bstart[bx];
            int ncol = b.near.col_ptr[bx + 1] - b.near.col_ptr[bx];
            double *rE = out + (size_t)(2 * i) * row_len;
            double *rH = out + (size_t)(2 * i + 1) * row_len;
            for (int c = 0; c < ncol; ++c) {
                int n = o.order[b.near.cols[b.near.col_ptr[bx] + c]];
                int64_t idx = b.near.val_ptr[bx] + (int64_t)row * ncol + c;
                cd A = b.near.A[idx], B = b.near.B[idx], C = b.near.C[idx], D = b.near.d(idx);
                rE[2 * n] = A.real();
                rE[2 * n + 1] = A.imag();
                rE[2 * (ne + n)] = -B.real();
                rE[2 * (ne + n) + 1] = -B.imag();
                rH[2 * n] = D.real();
                rH[2 * n + 1] = D.imag();
                rH[2 * (ne + n)] = C.real();
                rH[2 * (ne + n) + 1] = C.imag();
            }
        }
    });
}

sfmm_status sfmm_describe(const sfmm_ctx *ctx, int32_t body, int64_t *info, int32_t *trunc) {
    return guarded(const_cast<sfmm_ctx *>(ctx), [&] {
        const BodyHost &b = body_of(ctx, body);
        if (info) {
            info[0] = b.oct.nlev;
            info[1] = b.oct.nb;
            info[2] = b.oct.near_pairs;
            info[3] = b.oct.trans_pairs;
        }
        if (trunc) {
            for (int i = 0; i < 8 * 16; ++i) trunc[i] = 0;
            for (const RegionTree &rt : b.oct.regions) {
                if (rt.region >= 8) continue;
                for (size_t l = 0; l < rt.levels_L.size() && l < 16; ++l) trunc[rt.region * 16 + l] = rt.levels_L[l];
            }
        }
    });
}

sfmm_status sfmm_product_bytes(const sfmm_ctx *ctx, int32_t body, int64_t *bytes) {
    return guarded(const_cast<sfmm_ctx *>(ctx), [&] {
        if (!bytes) throw Error(SFMM_E_INVALID_ARG, "NULL output");
        const BodyHost &b = body_of(ctx, body);
        const int64_t cb = ctx->opt.precision == SFMM_PREC_FP64 ? 16 : 8;   // one stored complex number
        const int64_t ne = b.mesh.ne;
        int64_t col = 0;
        for (int i = 0; i < b.oct.nb; ++i) col += b.near.col_ptr[i + 1] - b.near.col_ptr[i];
        const int64_t planes = b.near.D.empty() ? 3 : 4;
        int64_t nearb = planes * cb * b.oct.near_pairs + 4 * col, xy = 2 * (2 * ne) * cb, pat = 0, lev = 0, trans = 0,
                interp = 0;
        for (size_t r = 0; r < b.oct.regions.size(); ++r) {
            const RegionTree &rt = b.oct.regions[r];
            const RegionTables &tb = b.tables[r];
            pat += cb * (int64_t)(tb.tx.size() + (tb.lossy ? tb.rx.size() : tb.tx.size()) + tb.nx.size());
            for (int l = 2; l <= b.oct.f; ++l) {
                const LevelBoxes &lv = rt.lev[l];
                const int64_t K = tb.samp[l].K;
                lev += 4 * cb * 2 * K * (int64_t)lv.key.size();
                std::vector<char> used(343, 0);
                for (int o : lv.il_off) used[o] = 1;
                int64_t nu = 0;
                for (char u : used) nu += u;
                trans += cb * K * nu;
                if (l >= 3)
                    interp += 4 * (int64_t)(tb.ipA[l].size() + tb.ipB[l].size() + tb.ipD[l].size()) +
                              cb * (int64_t)(tb.shift_up[l].size() + tb.shift_dn[l].size());
            }
        }
        bytes[0] = nearb;
        bytes[1] = xy;
        bytes[2] = pat;
        bytes[3] = lev;
        bytes[4] = trans;
        bytes[5] = interp;
        bytes[6] = nearb + xy + pat + lev + trans + interp;
        bytes[7] = 0;
    });
}

sfmm_status sfmm_profile(sfmm_ctx *ctx, int32_t enable, double *t, int64_t *n) {
    return guarded(ctx, [&] {
        if (!ctx) throw Error(SFMM_E_INVALID_ARG, "NULL context");
        StageTimes acc;
        for (auto &d : ctx->dev) {
            if (!d) continue;
            StageTimes s = d->times();
            for (int i = 0; i < 8; ++i) {
                acc.ms[i] += s.ms[i];
                acc.n[i] += s.n[i];
            }
            d->profile(enable != 0);
        }
        for (int i = 0; i < 8; ++i) {
            if (t) t[i] = acc.n[i] ? acc.ms[i] / acc.n[i] : 0.0;
            if (n) n[i] = acc.n[i];
        }
    });
}

void sfmm_guess_default_options(sfmm_guess_options *o) {
    if (!o) return;
    const GuessOptions d{};
    o->rank = d.rank;
    o->harmonics = d.harmonics;
    o->hidden = d.hidden;
    o->epochs = d.epochs;
    o->lr = d.lr;
    o->seed = d.seed;
    o->n_theta = d.n_theta;
    o->n_phi = d.n_phi;
}

sfmm_status sfmm_guess_fit(sfmm_ctx *ctx, int32_t body, int32_t n, const double *angles, const double *pol,
                           const void *x, const sfmm_guess_options *opt, double *final_loss, int32_t on_device) {
    return guarded(ctx, [&] {
        DeviceBody &d = dev_of(ctx, body);
        if (n <= 0 || !angles || !x) throw Error(SFMM_E_INVALID_ARG, "bad arguments");
        sfmm_guess_options go;
        sfmm_guess_default_options(&go);
        if (opt) go = *opt;
        GuessOptions g;
        g.rank = go.rank;
        g.harmonics = go.harmonics;
        g.hidden = go.hidden;
        g.epochs = go.epochs;
        g.lr = go.lr;
        g.seed = go.seed;
        g.n_theta = go.n_theta;
        g.n_phi = go.n_phi;
        const int N = 2 * ctx->bodies[body]->mesh.ne;
        const size_t bytes = (size_t)n * N * 2 * sizeof(double);
        Staged db(bytes);
        d.planewave_rhs(n, angles, pol, db.p);
        std::unique_ptr<Staged> dx;
        const void *xd = x;
        if (!on_device) {
            dx = std::make_unique<Staged>(bytes);
            copy_h2d(dx->p, x, bytes, d.stream());
            xd = dx->p;
        }
        if (ctx->guess.size() < ctx->bodies.size()) ctx->guess.resize(ctx->bodies.size());
        DeviceBody *dp = &d;   // the context's device bodies outlive its guesses
        auto gs = std::make_unique<Guess>(N, d.stream(), [dp](int m, const void *b, int nd, const double *dirs,
                                                              double *F) { dp->far_pattern(m, b, nd, dirs, F); });
        const double loss = gs->fit(n, angles, db.p, xd, g);
        ctx->guess[body] = std::move(gs);
        if (final_loss) *final_loss = loss;
    });
}

sfmm_status sfmm_guess_predict(sfmm_ctx *ctx, int32_t body, int32_t n, const double *angles, const double *pol,
                               void *x0, int32_t on_device) {
    return guarded(ctx, [&] {
        DeviceBody &d = dev_of(ctx, body);
        if (n <= 0 || !angles || !x0) throw Error(SFMM_E_INVALID_ARG, "bad arguments");
        if ((int)ctx->guess.size() <= body || !ctx->guess[body])
            throw Error(SFMM_E_INVALID_ARG, "learned guess is not trained for this body (call sfmm_guess_fit)");
        const int N = 2 * ctx->bodies[body]->mesh.ne;
        const size_t bytes = (size_t)n * N * 2 * sizeof(double);
        Staged db(bytes);
        d.planewave_rhs(n, angles, pol, db.p);
        if (on_device) {
            ctx->guess[body]->predict(n, angles, db.p, x0);
        } else {
            Staged dx(bytes);
            ctx->guess[body]->predict(n, angles, db.p, dx.p);
            copy_d2h(x0, dx.p, bytes, d.stream());
        }
    });
}

sfmm_status sfmm_span_predict(sfmm_ctx *ctx, int32_t body, int32_t n, const double *angles, const double *pol,
                              void *x0, int32_t on_device) {
    return guarded(ctx, [&] {
        DeviceBody &d = dev_of(ctx, body);
        if (n <= 0 || !angles || !x0) throw Error(SFMM_E_INVALID_ARG, "bad arguments");
        if ((int)ctx->guess.size() <= body || !ctx->guess[body])
            throw Error(SFMM_E_INVALID_ARG, "no training solutions for this body (call sfmm_guess_fit)");
        const int N = 2 * ctx->bodies[body]->mesh.ne;
        const size_t bytes = (size_t)n * N * 2 * sizeof(double);
        Staged db(bytes);
        d.planewave_rhs(n, angles, pol, db.p);
        auto product = [&](int r, const void *in, void *out) { d.matvec(r, in, out, SFMM_PART_ALL); };
        if (on_device) {
            ctx->guess[body]->span_predict(n, db.p, x0, product);
        } else {
            Staged dx(bytes);
            ctx->guess[body]->span_predict(n, db.p, dx.p, product);
            copy_d2h(x0, dx.p, bytes, d.stream());
        }
    });
}

sfmm_status sfmm_mlp_train(int32_t device, int32_t n_sizes, const int32_t *sizes, float *params, int32_t batch,
                           const float *X, const float *Y, int32_t steps, double lr, double *loss, float *grads,
                           float *out) {
    return guarded(nullptr, [&] {
        if (n_sizes < 2 || n_sizes > 16 || !sizes || !params || batch <= 0 || !X || !Y || steps < 0)
            throw Error(SFMM_E_INVALID_ARG, "bad arguments");
        std::vector<int> sz(sizes, sizes + n_sizes);
        check_device(device);
        use_device(device);
        Mlp net(sz, nullptr);
        net.set_params(params);
        const size_t nin = (size_t)batch * sz.front(), nout = (size_t)batch * sz.back();
        Staged dX(sizeof(float) * nin), dY(sizeof(float) * nout);
        copy_h2d(dX.p, X, sizeof(float) * nin, nullptr);
        copy_h2d(dY.p, Y, sizeof(float) * nout, nullptr);
        const float *fx = (const float *)dX.p, *fy = (const float *)dY.p;
        if (out) copy_d2h(out, net.forward(batch, fx), sizeof(float) * nout, nullptr);
        for (int32_t t = 0; t <= steps; ++t) {
            const double l = net.loss_grad(batch, fx, fy, loss != nullptr);
            if (loss) loss[t] = l;
            if (t == 0 && grads) net.get_grads(grads);
            if (t < steps) net.adam_step(lr);
        }
        if (steps > 0) net.get_params(params);
    });
}

}  // extern "C"
