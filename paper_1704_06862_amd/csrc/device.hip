// Device orchestration for gfx950 (MI355X): upload of the host tables, the
// batched MLFMM-accelerated PMCHWT product, the preconditioners and a
// lockstep batched flexible GMRES in FP64.  Kernels are in kernels.hpp.
//
// Data layout in HBM (internal order = finest boxes in colour/Morton order,
// canonical edge order inside a box; unknown u = 2p + {J, M~} of position p;
// right-hand side r of unknown u at u * R + r):
//   near matrix     per finest box, row-major [n_b][nc_b] planes A, B, C of
//                   complex T (block [[A,-B],[B,C]] per edge pair)
//   ILU(0) factors  per finest box, row-major [2 n_b][2 nc_b] complex T
//   patterns        per region, [n_edges_r][2][K_f] complex T (theta, phi)
//   level arrays    per region and level, [n_boxes][2][K_l][R] complex T
//   translations    per region and level, [343 offsets][K_l] complex T
//   Krylov vectors  FP64, [basis index][right-hand side][2E]
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "device.hpp"
#include "mfma.hpp"
#include "kernels.hpp"

// Scratch of the allocation-free far-field entry point (sfmm_rcs_noalloc):
// staging for the directions and the RCS values.  One copy per GPU, held
// until the process ends; every context on that GPU shares it, so calls that
// overlap on one GPU race.
constexpr size_t SFMM_SCRATCH_DOUBLES = 262144;   // 2 MiB
static __device__ __align__(256) double scratch[SFMM_SCRATCH_DOUBLES];

namespace sfmm {

#define HIPCHK(expr)                                                                             \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            throw Error(SFMM_E_DEVICE, std::string(#expr) + " failed: " + hipGetErrorString(e_)); \
    } while (0)

#define LAUNCHCHK() HIPCHK(hipGetLastError())

constexpr int MAXLEV = 21;
constexpr size_t LDS_LIMIT = 64 * 1024;
constexpr int BATCH = 64;        // right-hand sides per batched chunk
constexpr int TRANS_GRP_MIN_R = 16;  // sibling-grouped translation from this many RHS
// default plan: the batched near product (also inside the polynomial
// preconditioner) runs on the matrix cores from NEAR_MMA_MIN_R right-hand
// sides, aggregation, interpolation and receive from MMA_MIN_R (measured
// crossovers against the vector kernels on the 61,440- and 307,200-unknown
// spheres; below them the vector kernels are as fast or faster)
constexpr int NEAR_MMA_MIN_R = 3;
constexpr int MMA_MIN_R = 6;
constexpr int MMA_GATE_R = 2;    // the matrix-core kernels take any batch of at least this many RHS

void *device_alloc(size_t bytes) {
    void *p = nullptr;
    if (bytes == 0) bytes = 16;
    hipError_t e = hipMalloc(&p, bytes);
    if (e == hipErrorOutOfMemory)
        throw Error(SFMM_E_OOM, "device allocation of " + std::to_string(bytes) + " bytes failed");
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

size_t noalloc_scratch_doubles() { return SFMM_SCRATCH_DOUBLES; }

namespace {

// Device address of `scratch` on each GPU, looked up once per device with
// that device current (the host-side name of the array is not a device
// address).
std::mutex g_scratch_mutex;
std::map<int, double *> g_scratch_addr;

double *scratch_address(int device) {
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    auto it = g_scratch_addr.find(device);
    if (it != g_scratch_addr.end()) return it->second;
    void *p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_addr[device] = (double *)p;
    return (double *)p;
}

std::mutex g_capture_mutex;

inline unsigned nblocks(int64_t n, int bs = WG) { return (unsigned)((n + bs - 1) / bs); }

template <typename T>
cx<T> to_cx(cd v) {
    return {(T)v.real(), (T)v.imag()};
}

// largest candidate tile that divides R and satisfies fits(rt); 0 if none
template <typename F>
int pick_tile(int R, std::initializer_list<int> cands, F fits) {
    for (int rt : cands)
        if (R % rt == 0 && fits(rt)) return rt;
    return 0;
}

template <typename T>
class DeviceBodyT final : public DeviceBody {
  public:
    DeviceBodyT(const BodyHost &h, int device, void *stream, bool split, bool graphs, bool autotune, int kernel_plan,
                int verbose)
        : h_(h), split_(split), graphs_(graphs), autotune_(autotune), kernel_plan_(kernel_plan), verbose_(verbose) {
        HIPCHK(hipSetDevice(device));
        scratch_ = scratch_address(device);
        // a stream of our own stands in for the legacy default stream, which
        // cannot be captured; it is a blocking stream, so it stays ordered
        // with work on the default stream
        HIPCHK(hipStreamCreate(&own_stream_));
        set_stream(stream);
        const Mesh &m = h.mesh;
        const Octree &o = h.oct;
        ne_ = m.ne;
        nb_ = o.nb;
        f_ = o.f;
        colour_ptr_ = o.colour_ptr;
        pos_ = upload(o.pos);
        bstart_ = upload(o.bstart);
        near_col_ptr_ = upload(h.near.col_ptr);
        near_cols_ = upload(h.near.cols);
        near_val_ptr_ = upload(h.near.val_ptr);
        nA_ = upload_cx(h.near.A);
        nB_ = upload_cx(h.near.B);
        nC_ = upload_cx(h.near.C);
        gen_ = h.form != SFMM_FORM_PMCHWT;
        if (gen_) nD_ = upload_cx(h.near.D);
        // weight of the tangential parts: JMCFIE = (N parts) - (T parts)
        tang_ = h.form == SFMM_FORM_CNF ? cx<T>{0, 0} : cx<T>{-1, 0};
        precond_ = h.precond;
        if constexpr (std::is_same<T, float>::value) {
            if (precond_ == SFMM_PRECOND_POLY) {
                // bfloat16 copy of the blocks for the polynomial preconditioner
                // (a fixed approximation of the near-field inverse: half the
                // bytes of its products; GMRES still converges on Z itself)
                h16A_ = upload_bf16x2(h.near.A);
                h16B_ = upload_bf16x2(h.near.B);
                h16C_ = upload_bf16x2(h.near.C);
                if (gen_) h16D_ = upload_bf16x2(h.near.D);
            }
        }
        for (const cd &t : h.poly) inv_theta_.push_back(to_cx<T>(1.0 / t));
        if (!h.poly_dinv.empty()) dinv_ = upload_cx(h.poly_dinv);
        for (int b = 0; b < nb_; ++b) {
            max_ncol_ = std::max(max_ncol_, h.near.col_ptr[b + 1] - h.near.col_ptr[b]);
            max_nrow_ = std::max(max_nrow_, o.bstart[b + 1] - o.bstart[b]);
        }
        {
            // (box, row group) of every non-empty group of WAVES rows
            std::vector<int> grp;
            for (int b = 0; b < nb_; ++b)
                for (int rg = 0; rg * WAVES < o.bstart[b + 1] - o.bstart[b]; ++rg) {
                    grp.push_back(b);
                    grp.push_back(rg);
                }
            near_ngrp_ = (int)(grp.size() / 2);
            if (near_ngrp_ > 0) near_grp_ = upload(grp);
        }
        if constexpr (std::is_same<T, float>::value) build_mma_tiles(h);
        upload_edge_quadrature(m);
        if (!h.ilu.fwd_col_ptr.empty()) {
            fcol_ptr_ = upload(h.ilu.fwd_col_ptr);
            fcols_ = upload(h.ilu.fwd_cols);
            fptr_ = upload(h.ilu.fwd_ptr);
            fval_ = upload_cx(h.ilu.fwd);
            for (int b = 0; b < nb_; ++b)
                max_ilu_nc_ = std::max(max_ilu_nc_, h.ilu.fwd_col_ptr[b + 1] - h.ilu.fwd_col_ptr[b]);
        }
        if (!h.ilu.bwd_col_ptr.empty()) {
            bcol_ptr_ = upload(h.ilu.bwd_col_ptr);
            bcols_ = upload(h.ilu.bwd_cols);
            bptr_ = upload(h.ilu.bwd_ptr);
            bval_ = upload_cx(h.ilu.bwd);
            for (int b = 0; b < nb_; ++b)
                max_ilu_nc_ = std::max(max_ilu_nc_, h.ilu.bwd_col_ptr[b + 1] - h.ilu.bwd_col_ptr[b]);
        }
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
            {
                std::vector<int> eb(rt.edge_pos.size());
                for (int b = 0; b + 1 < (int)rt.edge_ptr.size(); ++b)
                    for (int e = rt.edge_ptr[b]; e < rt.edge_ptr[b + 1]; ++e) eb[e] = b;
                R.edge_box = upload(eb);
                R.ne = (int)eb.size();
            }
            for (int b = 0; b + 1 < (int)rt.edge_ptr.size(); ++b)
                R.max_ebox = std::max(R.max_ebox, rt.edge_ptr[b + 1] - rt.edge_ptr[b]);
            if (f_ >= 2) {
                R.tx = upload_cx(tb.tx);
                if (tb.lossy) R.rx = upload_cx(tb.rx);
                if (!tb.nx.empty()) R.nx = upload_cx(tb.nx);
                for (int l = 2; l <= f_; ++l) {
                    const Sampling &s = tb.samp[l];
                    const LevelBoxes &lv = rt.lev[l];
                    R.K[l] = s.K;
                    R.nth[l] = s.nth;
                    R.nph[l] = s.nph;
                    R.nbox[l] = (int)lv.key.size();
                    R.il_ptr[l] = upload(lv.il_ptr);
                    R.il_src[l] = upload(lv.il_src);
                    R.il_off[l] = upload(lv.il_off);
                    build_translation_groups(R, l, lv);
                    R.trans[l] = upload_cx(tb.trans[l]);
                    if (l >= 3) {
                        R.parent[l] = upload(lv.parent);
                        R.slot[l] = upload(lv.child_slot);
                        R.ipA[l] = upload_real(tb.ipA[l]);
                        R.ipB[l] = upload_real(tb.ipB[l]);
                        R.ipD[l] = upload_real(tb.ipD[l]);
                        const int np_p = tb.samp[l - 1].nph, np_c = s.nph;
                        std::vector<double> Dt((size_t)np_p * np_c);
                        for (int J = 0; J < np_p; ++J)
                            for (int jj = 0; jj < np_c; ++jj)
                                Dt[(size_t)jj * np_p + J] = tb.ipD[l][(size_t)J * np_c + jj];
                        R.ipDt[l] = upload_real(Dt);
                        R.sup[l] = upload_cx(tb.shift_up[l]);
                        R.sdn[l] = upload_cx(tb.shift_dn[l]);
                        if constexpr (std::is_same<T, float>::value) {
                            // phi stage with the child shift folded in, per (octant, parent theta row)
                            const int nt_p = tb.samp[l - 1].nth;
                            const size_t Kp = (size_t)nt_p * np_p;
                            std::vector<cd> up((size_t)8 * nt_p * np_p * np_c), dn(up.size());
                            for (int sl = 0; sl < 8; ++sl)
                                for (int I = 0; I < nt_p; ++I)
                                    for (int J = 0; J < np_p; ++J)
                                        for (int jj = 0; jj < np_c; ++jj) {
                                            const double d = tb.ipD[l][(size_t)J * np_c + jj];
                                            const size_t q = (size_t)sl * Kp + (size_t)I * np_p + J;
                                            up[(((size_t)sl * nt_p + I) * np_p + J) * np_c + jj] = d * tb.shift_up[l][q];
                                            dn[(((size_t)sl * nt_p + I) * np_c + jj) * np_p + J] = d * tb.shift_dn[l][q];
                                        }
                            R.Dup[l] = upload_cx(up);
                            R.Ddn[l] = upload_cx(dn);
                        }
                    }
                    if (l < f_) {
                        R.child_ptr[l] = upload(lv.child_ptr);
                        R.child_idx[l] = upload(lv.child_idx);
                    }
                }
            }
            regs_.push_back(R);
        }
        build_receive_all(o);
        HIPCHK(hipEventCreate(&ev0_));
        HIPCHK(hipEventCreate(&ev1_));
        for (auto &e : evs_) HIPCHK(hipEventCreate(&e));
        ensure_batch(1);
    }

    ~DeviceBodyT() override {
        clear_graphs();
        if (own_stream_) {
            (void)hipStreamSynchronize(own_stream_);
            (void)hipStreamDestroy(own_stream_);
        }
        for (void *p : batch_allocs_) device_free(p);
        for (void *p : krylov_allocs_) device_free(p);
        for (void *p : allocs_) device_free(p);
        if (ev0_) (void)hipEventDestroy(ev0_);
        if (ev1_) (void)hipEventDestroy(ev1_);
        if (pin_) (void)hipHostFree(pin_);
        for (auto &e : evs_)
            if (e) (void)hipEventDestroy(e);
    }

    void set_stream(void *s) override {
        const hipStream_t next = s ? (hipStream_t)s : own_stream_;
        if (next != stream_ && pin_off_ > 0 && stream_) {
            // the staging arena may still feed copies on the old stream
            HIPCHK(hipStreamSynchronize(stream_));
            pin_off_ = 0;
        }
        stream_ = next;
    }

    // Host -> device copy of a small host array (Krylov coefficients, active
    // lists) through a pinned staging arena, so the copy runs asynchronously
    // in stream order and the caller's array may change or go away as soon
    // as this returns.  The arena is reused from its start only after the
    // stream has drained.
    void stage_h2d(void *dst, const void *src, size_t bytes) {
        const size_t need = (bytes + 255) & ~(size_t)255;
        if (pin_off_ + need > pin_cap_) {
            HIPCHK(hipStreamSynchronize(stream_));
            pin_off_ = 0;
            if (need > pin_cap_) {
                if (pin_) HIPCHK(hipHostFree(pin_));
                pin_ = nullptr;
                pin_cap_ = std::max<size_t>(need, (size_t)1 << 20);
                HIPCHK(hipHostMalloc((void **)&pin_, pin_cap_, hipHostMallocDefault));
            }
        }
        std::memcpy(pin_ + pin_off_, src, bytes);
        HIPCHK(hipMemcpyAsync(dst, pin_ + pin_off_, bytes, hipMemcpyHostToDevice, stream_));
        pin_off_ += need;
    }
    void *stream() const override { return stream_; }
    void stream_synchronize() override { HIPCHK(hipStreamSynchronize(stream_)); }

    // ---- HIP graphs: one executable graph per (operation, batch size) ----
    enum GraphKind { G_PRODUCT = 0, G_PRECOND = 1, G_PREC_PRODUCT = 2 };

    void clear_graphs() {
        for (auto &kv : gexec_) (void)hipGraphExecDestroy(kv.second);
        gexec_.clear();
    }

    // Runs body() through a captured graph (captured on first use), or
    // directly while stage profiling is on or graphs are disabled.  body()
    // must only launch work on stream_ that reads and writes the fixed
    // internal buffers of batch size R.
    template <typename F>
    void run_graph(int kind, int R, F &&body) {
        if (!graphs_ || profiling_) {
            body();
            return;
        }
        const std::pair<int, int> key(kind, R);
        auto it = gexec_.find(key);
        if (it == gexec_.end()) {
            // first-time captures and instantiations run one at a time in the
            // process (bodies solved concurrently capture from several threads)
            std::lock_guard<std::mutex> lock(g_capture_mutex);
            HIPCHK(hipStreamBeginCapture(stream_, hipStreamCaptureModeThreadLocal));
            try {
                body();
            } catch (...) {
                hipGraph_t broken = nullptr;
                (void)hipStreamEndCapture(stream_, &broken);
                if (broken) (void)hipGraphDestroy(broken);
                throw;
            }
            hipGraph_t g = nullptr;
            HIPCHK(hipStreamEndCapture(stream_, &g));
            hipGraphExec_t ex = nullptr;
            const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            HIPCHK(e);
            it = gexec_.emplace(key, ex).first;
        }
        HIPCHK(hipGraphLaunch(it->second, stream_));
    }
    void profile(bool enable) override {
        profiling_ = enable;
        if (enable) times_ = StageTimes();
    }
    StageTimes times() const override { return times_; }
    int64_t device_bytes() const override { return bytes_; }

    // ---- kernel choice per batch size ----
    // Each stage with two implementations (vector kernel / matrix-core or
    // grouped kernel) is chosen per batch size R: by fixed thresholds, or,
    // with autotuning on, by timing both on the first batch of that size
    // (one stage at a time, the others at their current best).
    struct Plan {
        bool near_mma = false, agg_mma = false, interp_mma = false, trans_grp = false;
        bool interp_split = false;   // one RHS: theta and phi stages as separate whole-level launches
        bool overlap_trans = false;  // one RHS: coarsest phi stage and finer translations in one launch
        bool near_join = false;      // ... and the near product in the level-2 translation launch
        bool interp_fused = false;   // one RHS: downward phi and theta stages fused per level
    };
    static Plan default_plan(int R) {
        Plan p;
        p.near_mma = R >= NEAR_MMA_MIN_R && std::is_same<T, float>::value;
        p.agg_mma = p.interp_mma = R >= MMA_MIN_R && std::is_same<T, float>::value;
        p.trans_grp = R == 1 || R >= TRANS_GRP_MIN_R;
        p.interp_split = R == 1;
        p.overlap_trans = R == 1;
        p.near_join = R == 1;
        p.interp_fused = R == 1;
        return p;
    }
    void use_plan(int R) {
        if (kernel_plan_ & 1) {
            plan_.near_mma = (kernel_plan_ >> 1) & 1;
            plan_.agg_mma = (kernel_plan_ >> 2) & 1;
            plan_.interp_mma = (kernel_plan_ >> 3) & 1;
            plan_.trans_grp = (kernel_plan_ >> 4) & 1;
            plan_.interp_split = (kernel_plan_ >> 5) & 1;
            plan_.overlap_trans = (kernel_plan_ >> 7) & 1;
            plan_.near_join = (kernel_plan_ >> 8) & 1;
            plan_.interp_fused = (kernel_plan_ >> 9) & 1;
            return;
        }
        if (!autotune_) {
            plan_ = default_plan(R);
            return;
        }
        // one tuned plan per size class (exact below 16, multiples of 16 above)
        const int cls = R < 16 ? R : (R + 15) / 16 * 16;
        auto it = plans_.find(cls);
        if (it == plans_.end()) it = plans_.emplace(cls, tune(R)).first;
        plan_ = it->second;
    }
    float time_product(int R) {
        float best = 1e30f;
        for (int rep = 0; rep < 3; ++rep) {
            HIPCHK(hipEventRecord(ev0_, stream_));
            matvec_internal(xi_, yi_, R, SFMM_PART_ALL);
            HIPCHK(hipEventRecord(ev1_, stream_));
            HIPCHK(hipEventSynchronize(ev1_));
            float ms = 0;
            HIPCHK(hipEventElapsedTime(&ms, ev0_, ev1_));
            best = std::min(best, ms);
        }
        return best;
    }
    Plan tune(int R) {
        ensure_batch(R);
        const bool prof = profiling_;
        profiling_ = false;
        k_zero<T><<<nblocks((int64_t)2 * ne_ * R), WG, 0, stream_>>>(xi_, (int64_t)2 * ne_ * R);
        LAUNCHCHK();
        Plan best = default_plan(R);
        plan_ = best;
        float tbest = time_product(R);
        bool Plan::*fields[8] = {&Plan::near_mma,     &Plan::agg_mma,       &Plan::interp_mma, &Plan::trans_grp,
                                 &Plan::interp_split, &Plan::overlap_trans, &Plan::near_join, &Plan::interp_fused};
        for (bool Plan::*f : fields) {
            if (f == &Plan::interp_split || f == &Plan::overlap_trans || f == &Plan::near_join ||
                f == &Plan::interp_fused) {
                if (R != 1) continue;
            } else if (f != &Plan::trans_grp) {
                if (!std::is_same<T, float>::value || R < MMA_GATE_R) continue;
            }
            plan_ = best;
            plan_.*f = !(best.*f);
            const float t = time_product(R);
            if (t < tbest) {
                tbest = t;
                best = plan_;
            }
        }
        profiling_ = prof;
        if (verbose_)
            std::fprintf(stderr, "sfmm autotune R=%d: near %s, aggregate/receive %s, interpolation %s, translation %s "
                                 "(%.3f ms)\n",
                         R, best.near_mma ? "mfma" : "vector", best.agg_mma ? "mfma" : "vector",
                         best.interp_mma      ? "mfma"
                         : best.interp_fused ? "vector, fused downward stages"
                         : best.interp_split ? "vector, split stages"
                                             : "vector",
                         best.trans_grp ? "grouped" : "flat", tbest);
        return best;
    }

    // ---- batched products on internal T vectors [2E][R] ----
    template <bool POLY>
    void launch_near(int R, const cx<T> *x, cx<T> *y, cx<T> *acc, cx<T> inv_theta, int write_y) {
        if constexpr (std::is_same<T, float>::value) {
            if (plan_.near_mma && R >= MMA_GATE_R && ntiles_ > 0) {
                launch_near_mma<POLY>(R, x, y, acc, inv_theta, write_y);
                return;
            }
        }
        const int rt = pick_tile(R, {8, 4, 2, 1},
                                 [&](int t) { return (size_t)max_ncol_ * 2 * t * sizeof(cx<T>) <= LDS_LIMIT; });
        const bool lds = rt > 0;
        const int t = lds ? rt : 1;
        dim3 grid(nb_, (max_nrow_ + RW - 1) / RW, R / t);
        const size_t shm = lds ? (size_t)max_ncol_ * 2 * t * sizeof(cx<T>) : 0;
        // the polynomial preconditioner reads the bfloat16 copy of the blocks
        const bool h16 = POLY && h16A_ != nullptr;
#define SFMM_NEAR_H(RT_, L_, G_, H_)                                                                                 \
    k_near<T, RT_, L_, POLY, G_, H_><<<grid, RWG, shm, stream_>>>(R, bstart_, near_col_ptr_, near_cols_,              \
                                                                  near_val_ptr_, nA_, nB_, nC_, nD_, x, y, acc,     \
                                                                  inv_theta, write_y, POLY ? dinv_ : nullptr,       \
                                                                  h16A_, h16B_, h16C_, h16D_)
#define SFMM_NEAR_(RT_, L_, G_)                                    \
    do {                                                           \
        if constexpr (POLY && std::is_same<T, float>::value) {    \
            if (h16) SFMM_NEAR_H(RT_, L_, G_, true);               \
            else SFMM_NEAR_H(RT_, L_, G_, false);                  \
        } else {                                                   \
            SFMM_NEAR_H(RT_, L_, G_, false);                       \
        }                                                          \
    } while (0)
#define SFMM_NEAR(RT_, L_)                  \
    do {                                    \
        if (gen_) SFMM_NEAR_(RT_, L_, true);  \
        else SFMM_NEAR_(RT_, L_, false);      \
    } while (0)
        if (!lds) SFMM_NEAR(1, false);
        else if (t == 8) SFMM_NEAR(8, true);
        else if (t == 4) SFMM_NEAR(4, true);
        else if (t == 2) SFMM_NEAR(2, true);
        else SFMM_NEAR(1, true);
#undef SFMM_NEAR
#undef SFMM_NEAR_
#undef SFMM_NEAR_H
        LAUNCHCHK();
    }

    template <bool POLY>
    void launch_near_mma(int R, const cx<float> *x, cx<float> *y, cx<float> *acc, cx<float> inv_theta,
                         int write_y) {
        const int nt = (R + 15) / 16;
        const unsigned ng = (unsigned)((ntiles_ + 7) / 8 * 8);
#define SFMM_NMMA_(NT_, S_, G_)                                                                                 \
    k_near_mma<NT_, S_, POLY, G_><<<ng, 64 * MMA_WAVES, 0, stream_>>>(R, tile_box_, tile_row0_, tile_step_, bstart_, \
                                                                    near_col_ptr_, near_cols_, tvals_, nsteps_, x,  \
                                                                    y, acc, inv_theta, write_y,                    \
                                                                    POLY ? dinv_ : nullptr, ntiles_)
#define SFMM_NMMA(NT_, S_)                  \
    do {                                    \
        if (gen_) SFMM_NMMA_(NT_, S_, true);  \
        else SFMM_NMMA_(NT_, S_, false);      \
    } while (0)
        if (POLY && !ptvals_) throw Error(SFMM_E_DEVICE, "polynomial preconditioner tiles missing");
        if (POLY) {
            // the polynomial preconditioner: bfloat16 tiles of its own
            const unsigned pg = (unsigned)((pntiles_ + 7) / 8 * 8);
#define SFMM_PMMA_(NT_, G_)                                                                                        \
    k_near_mma<NT_, true, true, G_><<<pg, 64 * MMA_WAVES, 0, stream_>>>(R, ptile_box_, ptile_row0_, ptile_step_,  \
                                                                        bstart_, near_col_ptr_, near_cols_,       \
                                                                        ptvals_, pnsteps_, x, y, acc, inv_theta,  \
                                                                        write_y, dinv_, pntiles_)
#define SFMM_PMMA(NT_)                  \
    do {                                \
        if (gen_) SFMM_PMMA_(NT_, true);  \
        else SFMM_PMMA_(NT_, false);      \
    } while (0)
            if (nt == 1) SFMM_PMMA(1);
            else if (nt == 2) SFMM_PMMA(2);
            else if (nt == 3) SFMM_PMMA(3);
            else SFMM_PMMA(4);
#undef SFMM_PMMA
#undef SFMM_PMMA_
        } else if (split_) {
            if (nt == 1) SFMM_NMMA(1, true);
            else if (nt == 2) SFMM_NMMA(2, true);
            else if (nt == 3) SFMM_NMMA(3, true);
            else SFMM_NMMA(4, true);
        } else {
            if (nt == 1) SFMM_NMMA(1, false);
            else if (nt == 2) SFMM_NMMA(2, false);
            else if (nt == 3) SFMM_NMMA(3, false);
            else SFMM_NMMA(4, false);
        }
#undef SFMM_NMMA
#undef SFMM_NMMA_
        LAUNCHCHK();
    }

    // Near-field matrix in matrix-core tile order (see k_near_mma): tiles of
    // 16 rows of one box, K steps of 4 (FP32) or 32 (bf16 split) columns.
    void build_mma_tiles(const BodyHost &h) {
        build_product_tiles(h);
        if (precond_ == SFMM_PRECOND_POLY) build_poly_tiles(h);
    }

    // bfloat16 tiles of the blocks for the polynomial preconditioner's
    // matrix-core products: K steps of 32 columns, eight (PMCHWT: six)
    // compact planes (A, B, C[, D]) x (re, im), 8 bf16 per lane, each value
    // rounded to nearest even through FP32
    void build_poly_tiles(const BodyHost &h) {
        const Octree &o = h.oct;
        const NearMatrix &Z = h.near;
        std::vector<int> tbox, trow0;
        std::vector<int64_t> tstep{0};
        for (int b = 0; b < nb_; ++b) {
            const int nrow = o.bstart[b + 1] - o.bstart[b], ncol = Z.col_ptr[b + 1] - Z.col_ptr[b];
            const int nks = (ncol + 31) / 32;
            for (int row0 = 0; row0 < nrow; row0 += 16) {
                tbox.push_back(b);
                trow0.push_back(row0);
                tstep.push_back(tstep.back() + nks);
            }
        }
        if (tbox.empty() || tstep.back() == 0) return;
        pntiles_ = (int)tbox.size();
        pnsteps_ = tstep.back();
        const std::vector<cd> *mats[4] = {&Z.A, &Z.B, &Z.C, &Z.D};
        const int np = Z.D.empty() ? 3 : 4;
        auto rne = [](double v) {
            const float f = (float)v;
            uint32_t u;
            std::memcpy(&u, &f, 4);
            u += 0x7fffu + ((u >> 16) & 1u);
            return (uint16_t)(u >> 16);
        };
        std::vector<uint16_t> V((size_t)2 * np * pnsteps_ * 64 * 8, 0);
        for (int t = 0; t < pntiles_; ++t) {
            const int b = tbox[t], row0 = trow0[t];
            const int nrow = o.bstart[b + 1] - o.bstart[b], ncol = Z.col_ptr[b + 1] - Z.col_ptr[b];
            for (int64_t st = tstep[t]; st < tstep[t + 1]; ++st) {
                const int s = (int)(st - tstep[t]);
                for (int lane = 0; lane < 64; ++lane)
                    for (int e = 0; e < 8; ++e) {
                        const int row = row0 + lane % 16, col = 32 * s + 8 * (lane / 16) + e;
                        if (row >= nrow || col >= ncol) continue;
                        const int64_t idx = Z.val_ptr[b] + (int64_t)row * ncol + col;
                        for (int m = 0; m < np; ++m) {
                            const cd v = (*mats[m])[idx];
                            V[((((size_t)(2 * m) * pnsteps_ + st) * 64) + lane) * 8 + e] = rne(v.real());
                            V[((((size_t)(2 * m + 1) * pnsteps_ + st) * 64) + lane) * 8 + e] = rne(v.imag());
                        }
                    }
            }
        }
        ptile_box_ = upload(tbox);
        ptile_row0_ = upload(trow0);
        ptile_step_ = upload(tstep);
        ptvals_ = upload(V);
    }

    void build_product_tiles(const BodyHost &h) {
        const Octree &o = h.oct;
        const NearMatrix &Z = h.near;
        const int KS = split_ ? 32 : 4;
        std::vector<int> tbox, trow0;
        std::vector<int64_t> tstep{0};
        for (int b = 0; b < nb_; ++b) {
            const int nrow = o.bstart[b + 1] - o.bstart[b], ncol = Z.col_ptr[b + 1] - Z.col_ptr[b];
            const int nks = (ncol + KS - 1) / KS;
            for (int row0 = 0; row0 < nrow; row0 += 16) {
                tbox.push_back(b);
                trow0.push_back(row0);
                tstep.push_back(tstep.back() + nks);
            }
        }
        ntiles_ = (int)tbox.size();
        nsteps_ = tstep.back();
        if (ntiles_ == 0 || nsteps_ == 0) {
            ntiles_ = 0;
            return;
        }
        tile_box_ = upload(tbox);
        tile_row0_ = upload(trow0);
        tile_step_ = upload(tstep);
        const std::vector<cd> *mats[4] = {&Z.A, &Z.B, &Z.C, &Z.D};
        const int np = Z.D.empty() ? 3 : 4;   // planes: the general block adds D
        if (!split_) {
            std::vector<cx<float>> V((size_t)np * nsteps_ * 64, cx<float>{0, 0});
            for (int t = 0; t < ntiles_; ++t) {
                const int b = tbox[t], row0 = trow0[t];
                const int nrow = o.bstart[b + 1] - o.bstart[b], ncol = Z.col_ptr[b + 1] - Z.col_ptr[b];
                for (int64_t st = tstep[t]; st < tstep[t + 1]; ++st) {
                    const int s = (int)(st - tstep[t]);
                    for (int lane = 0; lane < 64; ++lane) {
                        const int row = row0 + lane % 16, col = 4 * s + lane / 16;
                        if (row >= nrow || col >= ncol) continue;
                        const int64_t idx = Z.val_ptr[b] + (int64_t)row * ncol + col;
                        for (int m = 0; m < np; ++m)
                            V[((size_t)m * nsteps_ + st) * 64 + lane] = to_cx<float>((*mats[m])[idx]);
                    }
                }
            }
            tvals_ = upload(V);
        } else {
            // twelve (or sixteen) planes (A, B, C[, D]) x (re hi, re lo, im hi, im lo), 8 bf16 per lane
            std::vector<uint16_t> V((size_t)4 * np * nsteps_ * 64 * 8, 0);
            auto bf = [](double v, uint16_t &hi, uint16_t &lo) {
                auto rne = [](float f) {
                    uint32_t u;
                    std::memcpy(&u, &f, 4);
                    u += 0x7fffu + ((u >> 16) & 1u);
                    return (uint16_t)(u >> 16);
                };
                auto back = [](uint16_t b) {
                    const uint32_t u = (uint32_t)b << 16;
                    float f;
                    std::memcpy(&f, &u, 4);
                    return (double)f;
                };
                hi = rne((float)v);
                lo = rne((float)(v - back(hi)));
            };
            for (int t = 0; t < ntiles_; ++t) {
                const int b = tbox[t], row0 = trow0[t];
                const int nrow = o.bstart[b + 1] - o.bstart[b], ncol = Z.col_ptr[b + 1] - Z.col_ptr[b];
                for (int64_t st = tstep[t]; st < tstep[t + 1]; ++st) {
                    const int s = (int)(st - tstep[t]);
                    for (int lane = 0; lane < 64; ++lane)
                        for (int e = 0; e < 8; ++e) {
                            const int row = row0 + lane % 16, col = 32 * s + 8 * (lane / 16) + e;
                            if (row >= nrow || col >= ncol) continue;
                            const int64_t idx = Z.val_ptr[b] + (int64_t)row * ncol + col;
                            for (int m = 0; m < np; ++m) {
                                const cd v = (*mats[m])[idx];
                                uint16_t q[4];
                                bf(v.real(), q[0], q[1]);
                                bf(v.imag(), q[2], q[3]);
                                for (int c = 0; c < 4; ++c)
                                    V[((((size_t)(4 * m + c) * nsteps_ + st) * 64) + lane) * 8 + e] = q[c];
                            }
                        }
                }
            }
            tvals_ = upload(V);
        }
    }

  private:
    struct Reg;

  public:
    void aggregate_region(Reg &G, int R, const cx<T> *x) {
        const int f = f_;
        if constexpr (std::is_same<T, float>::value) {
            if (plan_.agg_mma && R >= MMA_GATE_R) {
                aggregate_mma(G, R, x);
                return;
            }
        }
        launch_aggregate(agg(G), AggRegion<T>{}, R, x);
    }
    AggRegion<T> agg(const Reg &G) const {
        return AggRegion<T>{G.K[f_], G.nbf, G.edge_ptr, G.edge_pos, G.edge_sign, G.tx, G.et, G.S[f_]};
    }
    void launch_aggregate(const AggRegion<T> &a, const AggRegion<T> &b, int R, const cx<T> *x) {
        const int nwg = a.nbf + b.nbf;
        if (nwg <= 0) return;
        const int ech = std::max(1, 2048 / R);
        const int kmax = std::max(a.K, b.nbf > 0 ? b.K : 0);
        const int bs = (int)std::min<int64_t>(1024, (((int64_t)kmax * R + 63) / 64) * 64);
        const size_t shm = (size_t)2 * ech * R * sizeof(cx<T>);
        k_aggregate<T><<<nwg, bs, shm, stream_>>>(a, b, R, ech, x);
        LAUNCHCHK();
    }
    // Aggregation of every region: with the vector kernel, two regions per
    // launch (the larger-K region first).
    void aggregate_all(int R, const cx<T> *x) {
        bool mma = false;
        if constexpr (std::is_same<T, float>::value) mma = plan_.agg_mma && R >= MMA_GATE_R;
        if (mma) {
            for (Reg &G : regs_) aggregate_region(G, R, x);
            return;
        }
        for (size_t i = 0; i < regs_.size(); i += 2) {
            AggRegion<T> a = agg(regs_[i]), b = i + 1 < regs_.size() ? agg(regs_[i + 1]) : AggRegion<T>{};
            if (b.nbf > 0 && b.K > a.K) std::swap(a, b);
            launch_aggregate(a, b, R, x);
        }
    }

    Rcv1Region<T> rcv1(const Reg &G) const {
        Rcv1Region<T> r{};
        r.ne = G.ne;
        r.K = G.K[f_];
        r.nwaves = (G.ne + 7) / 8;
        r.edge_box = G.edge_box;
        r.edge_pos = G.edge_pos;
        r.edge_sign = G.edge_sign;
        r.tab = G.lossy ? G.rx : G.tx;
        r.nx = G.nx;
        r.conj = G.lossy ? 0 : 1;
        r.inv_et = G.inv_et;
        r.G = G.G[f_];
        return r;
    }
    // The single-RHS receive of all regions as one launch: every internal
    // position's contributions (region, entry), region order.  Left unset
    // (one launch per region) for more than RCV_MAXREG regions or an odd
    // direction count.
    void build_receive_all(const Octree &o) {
        if (f_ < 2 || regs_.empty() || regs_.size() > (size_t)RCV_MAXREG) return;
        for (const Reg &G : regs_)
            if (G.K[f_] % 2 || G.ne >= (1 << RCV_REG_SHIFT)) return;
        std::vector<int> ptr(ne_ + 1, 0);
        for (const RegionTree &rt : o.regions)
            for (int p : rt.edge_pos) ++ptr[p + 1];
        int maxc = 0;
        for (int p = 0; p < ne_; ++p) {
            maxc = std::max(maxc, ptr[p + 1]);
            ptr[p + 1] += ptr[p];
        }
        std::vector<int> ent(ptr[ne_]), fill(ptr.begin(), ptr.end() - 1);
        for (size_t ri = 0; ri < o.regions.size(); ++ri) {
            const std::vector<int> &pos = o.regions[ri].edge_pos;
            for (size_t ie = 0; ie < pos.size(); ++ie) ent[fill[pos[ie]]++] = (int)ri << RCV_REG_SHIFT | (int)ie;
        }
        std::vector<Rcv1Region<T>> desc;
        for (const Reg &G : regs_) {
            desc.push_back(rcv1(G));
            desc.back().G = nullptr;   // per-batch buffer: passed at launch
        }
        rcv_all_.npos = ne_;
        rcv_all_.maxc = maxc;
        rcv_all_.ptr = upload(ptr);
        rcv_all_.ent = upload(ent);
        rcv_all_.reg = upload(desc);
    }
    void launch_receive1(const Rcv1Region<T> &a, cx<T> *y) {
        if (a.nwaves <= 0) return;
        const unsigned grid = nblocks(a.nwaves, WAVES);
        if (gen_) k_receive1<T, true><<<grid, WG, 0, stream_>>>(a, tang_.x, y);
        else k_receive1<T, false><<<grid, WG, 0, stream_>>>(a, tang_.x, y);
        LAUNCHCHK();
    }
    // Receive of every region: one launch for all of them at one RHS (when
    // the merged table was built), otherwise one launch each, in region
    // order (they add into the same entries of y).
    void receive_all(int R, cx<T> *y) {
        if (R == 1 && rcv_all_.reg) {
            Rcv1All<T> ra = rcv_all_;
            for (size_t i = 0; i < regs_.size(); ++i) ra.G[i] = regs_[i].G[f_];
            const unsigned grid = nblocks((ra.npos + 7) / 8, WAVES);
            if (gen_) k_receive1_all<T, true><<<grid, WG, 0, stream_>>>(ra, tang_.x, y);
            else k_receive1_all<T, false><<<grid, WG, 0, stream_>>>(ra, tang_.x, y);
            LAUNCHCHK();
            return;
        }
        for (Reg &G : regs_) receive_region(G, R, y);
    }
    void receive_region(Reg &G, int R, cx<T> *y) {
        const int f = f_;
        if constexpr (std::is_same<T, float>::value) {
            if (plan_.agg_mma && R >= MMA_GATE_R) {
                receive_mma(G, R, y);
                return;
            }
        }
        const T tg = tang_.x;
        if (R == 1 && G.K[f] % 2 == 0) {
            launch_receive1(rcv1(G), y);
            return;
        }
        const int rt = pick_tile(R, {8, 4, 2, 1}, [](int) { return true; });
        dim3 grid(G.nbf, R / rt);
#define SFMM_RECV_(RT_, LO_, N_)                                                                              \
    k_receive<T, RT_, LO_, N_><<<grid, WG, 0, stream_>>>(G.K[f], R, G.edge_ptr, G.edge_pos, G.edge_sign, G.tx, \
                                                         G.rx, G.nx, G.inv_et, tg, G.G[f], y)
#define SFMM_RECV(RT_)                       \
    if (G.lossy) {                           \
        if (gen_) SFMM_RECV_(RT_, true, true);   \
        else SFMM_RECV_(RT_, true, false);       \
    } else {                                 \
        if (gen_) SFMM_RECV_(RT_, false, true);  \
        else SFMM_RECV_(RT_, false, false);      \
    }
        if (rt == 8) {
            SFMM_RECV(8)
        } else if (rt == 4) {
            SFMM_RECV(4)
        } else if (rt == 2) {
            SFMM_RECV(2)
        } else {
            SFMM_RECV(1)
        }
#undef SFMM_RECV
#undef SFMM_RECV_
        LAUNCHCHK();
    }

    // y = Z x: the near product, then per stage every region's far-field
    // work (aggregation, upward pass, translation, downward pass, receive),
    // all on the library stream.
    void matvec_internal(const cx<T> *x, cx<T> *y, int R, int parts) {
        const int64_t NR = (int64_t)2 * ne_ * R;
        const bool far = (parts & SFMM_PART_FAR) && f_ >= 2;
        const bool overlap = far && !profiling_ && overlap_ok(R);
        // the near product may wait for that shared launch: y is not touched
        // before it, and the receive step adds to y after it
        const bool near_joined = overlap && (parts & SFMM_PART_NEAR) && near_join_ok(R);
        mark(0);
        if (parts & SFMM_PART_NEAR) {
            if (!near_joined) launch_near<false>(R, x, y, nullptr, cx<T>{0, 0}, 1);
        } else {
            k_zero<T><<<nblocks(NR), WG, 0, stream_>>>(y, NR);
            LAUNCHCHK();
        }
        mark(1);
        if (far) {
            aggregate_all(R, x);
            if (overlap) {
                // stage timing keeps the upward pass and the translation apart
                up_and_translate_overlapped(R, near_joined ? x : nullptr, y);
            } else {
                mark(2);
                for (int l = f_; l >= 3; --l) upward_level(l, R);
                mark(3);
                translate_all(R);
            }
            mark(4);
            for (int l = 3; l <= f_; ++l) downward_level(l, R);
            mark(5);
            receive_all(R, y);
        } else {
            mark(2);
            mark(3);
            mark(4);
            mark(5);
        }
        mark(6);
        if (profiling_) collect_matvec(R);
    }

    // Sibling groups for k_translate_grp: boxes sharing a parent key, the union
    // of their interaction lists as candidates, and per (candidate, octant)
    // the translation offset id or -1 when the pair is not in that list.
    void build_translation_groups(Reg &R, int l, const LevelBoxes &lv) {
        const int nbox = (int)lv.key.size();
        std::vector<std::array<int, 4>> order(nbox);   // parent key, box
        for (int b = 0; b < nbox; ++b) order[b] = {lv.key[b][0] >> 1, lv.key[b][1] >> 1, lv.key[b][2] >> 1, b};
        std::sort(order.begin(), order.end());
        std::vector<int> dst, cptr{0}, csrc;
        std::vector<int> coff;
        for (int i = 0; i < nbox;) {
            int j = i;
            while (j < nbox && order[j][0] == order[i][0] && order[j][1] == order[i][1] && order[j][2] == order[i][2])
                ++j;
            int d8[8] = {-1, -1, -1, -1, -1, -1, -1, -1};
            std::vector<int> cand;
            for (int q = i; q < j; ++q) {
                const int b = order[q][3];
                const auto &kk = lv.key[b];
                d8[(kk[0] & 1) * 4 + (kk[1] & 1) * 2 + (kk[2] & 1)] = b;
                for (int e = lv.il_ptr[b]; e < lv.il_ptr[b + 1]; ++e) cand.push_back(lv.il_src[e]);
            }
            std::sort(cand.begin(), cand.end());
            cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
            const size_t base = coff.size();
            coff.resize(base + cand.size() * 8, -1);
            for (int slot = 0; slot < 8; ++slot) {
                const int b = d8[slot];
                if (b < 0) continue;
                for (int e = lv.il_ptr[b]; e < lv.il_ptr[b + 1]; ++e) {
                    const size_t ci = std::lower_bound(cand.begin(), cand.end(), lv.il_src[e]) - cand.begin();
                    coff[base + ci * 8 + slot] = lv.il_off[e];
                }
            }
            for (int slot = 0; slot < 8; ++slot) dst.push_back(d8[slot]);
            csrc.insert(csrc.end(), cand.begin(), cand.end());
            cptr.push_back((int)csrc.size());
            i = j;
        }
        R.ngrp[l] = (int)cptr.size() - 1;
        R.grp_dst[l] = upload(dst);
        R.cand_ptr[l] = upload(cptr);
        R.cand_src[l] = upload(csrc);
        R.cand_off[l] = upload(coff);
    }

    void aggregate_mma(Reg &G, int R, const cx<float> *x) {
        const int f = f_, K = G.K[f], nmt = (K + 15) / 16, nt = (R + 15) / 16;
        dim3 grid(G.nbf, (nmt + 3) / 4);
#define SFMM_AGG(NT_)                                                                                               \
    k_aggregate_mma<NT_><<<grid, 256, 0, stream_>>>(K, R, nmt, G.edge_ptr, G.edge_pos, G.edge_sign, G.tx, G.et, x, \
                                                    G.S[f])
        if (nt == 1) SFMM_AGG(1);
        else if (nt == 2) SFMM_AGG(2);
        else if (nt == 3) SFMM_AGG(3);
        else SFMM_AGG(4);
#undef SFMM_AGG
        LAUNCHCHK();
    }

    // PMCHWT: one pass (MODE 0).  JMCFIE: the RWG pass (MODE 1) and the pass
    // of the rotated test functions (MODE 2, their table given as the
    // transmit table for real k, as the receive table otherwise); CNF: MODE 2.
    void receive_mma(Reg &G, int R, cx<float> *y) {
        const int f = f_, K = G.K[f], nt = (R + 15) / 16;
        dim3 grid(G.nbf, (G.max_ebox + 15) / 16);
        const float tg = tang_.x;
#define SFMM_RCV_(NT_, L_, MD_, TX_, RX_)                                                                          \
    k_receive_mma<NT_, L_, MD_><<<grid, 64 * MMA_WAVES, 0, stream_>>>(K, R, G.edge_ptr, G.edge_pos, G.edge_sign,  \
                                                                      TX_, RX_, G.inv_et, tg, G.G[f], y)
#define SFMM_RCV(L_, MD_, TX_, RX_)                     \
    do {                                                \
        if (nt == 1) SFMM_RCV_(1, L_, MD_, TX_, RX_);   \
        else if (nt == 2) SFMM_RCV_(2, L_, MD_, TX_, RX_); \
        else if (nt == 3) SFMM_RCV_(3, L_, MD_, TX_, RX_); \
        else SFMM_RCV_(4, L_, MD_, TX_, RX_);           \
    } while (0)
        if (!gen_) {
            if (G.lossy) SFMM_RCV(true, 0, G.tx, G.rx);
            else SFMM_RCV(false, 0, G.tx, G.rx);
        } else {
            if (tg != 0.f) {
                if (G.lossy) SFMM_RCV(true, 1, G.tx, G.rx);
                else SFMM_RCV(false, 1, G.tx, G.rx);
                LAUNCHCHK();
            }
            if (G.lossy) SFMM_RCV(true, 2, nullptr, G.nx);
            else SFMM_RCV(false, 2, G.nx, nullptr);
        }
#undef SFMM_RCV
#undef SFMM_RCV_
        LAUNCHCHK();
    }

    // matrix-core interpolation: sizes within 4 tiles of 16 (theta pairs and phi)
    // fewer than four 256-thread workgroups per CU: launch 64-thread ones
    static bool small_grid(int64_t items) { return nblocks(items) < 4 * 256; }

    // single-RHS split stages: the matrices of the transition l -> l - 1 fit in LDS
    bool split_ok(const Reg &G, int l, int R) const {
        const size_t th = (size_t)2 * G.nth[l - 1] * G.nth[l] * sizeof(T), ph = (size_t)G.nph[l - 1] * G.nph[l] * sizeof(T);
        return plan_.interp_split && R == 1 && G.tmp && G.nph[l] % 2 == 0 && G.nph[l - 1] % 2 == 0 &&
               th <= LDS_LIMIT && ph <= LDS_LIMIT;
    }

    // single-RHS fused downward transitions l - 1 -> l: one azimuth pair per
    // workgroup must fit LDS
    bool fused_ok(int l, int R) const {
        if (!plan_.interp_fused || R != 1 || (int)regs_.size() > SPLIT_MAXJOB) return false;
        for (const Reg &G : regs_)
            if (G.nph[l] % 2 || fused_dn_lds<T>(G.nth[l], G.nth[l - 1], G.nph[l - 1], 1) > LDS_LIMIT) return false;
        return true;
    }
    // azimuth-pair chunks per (child, component): about 2,048 workgroups per launch
    JobList<FusedDnJob<T>> fused_dn_jobs(int l, size_t &shm) {
        JobList<FusedDnJob<T>> jl{};
        int64_t groups = 0;
        for (Reg &G : regs_) groups += (int64_t)G.nbox[l] * 2;
        const int want = (int)std::max<int64_t>(1, (2048 + groups - 1) / groups);
        shm = 0;
        for (Reg &G : regs_) {
            const int nth_c = G.nth[l], nph_c = G.nph[l], nth_p = G.nth[l - 1], nph_p = G.nph[l - 1];
            const int h = nph_c / 2;
            int cols = (h + std::min(want, h) - 1) / std::min(want, h);
            while (cols > 1 && fused_dn_lds<T>(nth_c, nth_p, nph_p, cols) > LDS_LIMIT) --cols;
            const int nchunk = (h + cols - 1) / cols;
            shm = std::max(shm, fused_dn_lds<T>(nth_c, nth_p, nph_p, cols));
            add_job(jl, FusedDnJob<T>{G.nbox[l], nth_c, nph_c, nth_p, nph_p, cols, G.ipA[l], G.ipB[l], G.ipD[l],
                                      G.parent[l], G.slot[l], G.sdn[l], G.G[l - 1], G.G[l]},
                    (int64_t)G.nbox[l] * 2 * nchunk, 1);
        }
        return jl;
    }

    bool interp_mma_ok(const Reg &G, int l, int R) const {
        return plan_.interp_mma && R >= MMA_GATE_R && G.Dup[l] && 2 * G.nth[l - 1] <= 64 && 2 * G.nth[l] <= 64 && G.nph[l - 1] <= 64 &&
               G.nph[l] <= 64;
    }

    void upward_mma(Reg &G, int l, int R) {
        const int nt = (R + 15) / 16;
        const int nth_c = G.nth[l], nph_c = G.nph[l], nth_p = G.nth[l - 1], nph_p = G.nph[l - 1];
        const int ipb = mma_rows_per_wg(nph_p);
        const unsigned g1 = (unsigned)G.nbox[l] * 2, g2 = (unsigned)G.nbox[l - 1] * 2 * ((nth_p + ipb - 1) / ipb);
#define SFMM_UPM(NT_)                                                                                                \
    k_up_theta_mma<NT_><<<g1, 256, 0, stream_>>>(R, nth_c, nph_c, nth_p, G.ipA[l], G.ipB[l], G.S[l], G.tmp);         \
    LAUNCHCHK();                                                                                                     \
    k_up_phi_mma<NT_><<<g2, 256, 0, stream_>>>(R, nth_p, nph_p, nph_c, G.Dup[l], G.child_ptr[l - 1],                \
                                               G.child_idx[l - 1], G.slot[l], G.tmp, G.S[l - 1]);                    \
    LAUNCHCHK()
        if (nt == 1) { SFMM_UPM(1); }
        else if (nt == 2) { SFMM_UPM(2); }
        else if (nt == 3) { SFMM_UPM(3); }
        else { SFMM_UPM(4); }
#undef SFMM_UPM
    }

    void downward_mma(Reg &G, int l, int R) {
        const int nt = (R + 15) / 16;
        const int nth_c = G.nth[l], nph_c = G.nph[l], nth_p = G.nth[l - 1], nph_p = G.nph[l - 1];
        const int ipb = mma_rows_per_wg(nph_c);
        const unsigned g1 = (unsigned)G.nbox[l] * 2 * ((nth_p + ipb - 1) / ipb), g2 = (unsigned)G.nbox[l] * 2;
#define SFMM_DNM(NT_)                                                                                              \
    k_dn_phi_mma<NT_><<<g1, 256, 0, stream_>>>(R, nth_p, nph_p, nph_c, G.Ddn[l], G.parent[l], G.slot[l],            \
                                               G.G[l - 1], G.tmp);                                                 \
    LAUNCHCHK();                                                                                                   \
    k_dn_theta_mma<NT_><<<g2, 256, 0, stream_>>>(R, nth_c, nph_c, nth_p, G.ipA[l], G.ipB[l], G.tmp, G.G[l]);        \
    LAUNCHCHK()
        if (nt == 1) { SFMM_DNM(1); }
        else if (nt == 2) { SFMM_DNM(2); }
        else if (nt == 3) { SFMM_DNM(3); }
        else { SFMM_DNM(4); }
#undef SFMM_DNM
    }

    // job table of the grouped single-RHS translation: every region, levels
    // lmin..lmax
    TransGroups<T> trans_groups(int lmin, int lmax) const {
        TransGroups<T> tg{};
        int e = 0, nblk = 0;
        for (const Reg &G : regs_)
            for (int l = lmin; l <= lmax; ++l, ++e) {
                tg.blk0[e] = nblk;
                tg.K[e] = G.K[l];
                tg.nkc[e] = (G.K[l] + 63) / 64;
                tg.grp_dst[e] = G.grp_dst[l];
                tg.cand_ptr[e] = G.cand_ptr[l];
                tg.cand_src[e] = G.cand_src[l];
                tg.cand_off[e] = G.cand_off[l];
                tg.trans[e] = G.trans[l];
                tg.S[e] = G.S[l];
                tg.G[e] = G.G[l];
                nblk += G.ngrp[l] * tg.nkc[e];
            }
        tg.nlev = e;
        tg.blk0[e] = nblk;
        tg.nblk = nblk;
        return tg;
    }

    // One RHS, three or more levels: the coarsest upward phi stage shares a
    // launch with the translations of the finer levels (which only need the
    // finer levels' outgoing patterns); level 2 is translated after it.
    bool overlap_ok(int R) const {
        return R == 1 && plan_.trans_grp && plan_.overlap_trans && f_ >= 3 && split_all(3, R) &&
               (int)regs_.size() * (f_ - 1) <= TRANS_MAXJOB;
    }
    bool near_join_ok(int R) const {
        return R == 1 && plan_.near_join && near_ngrp_ > 0 &&
               (size_t)max_ncol_ * 2 * sizeof(cx<T>) <= LDS_LIMIT;
    }
    // x != nullptr: the near product y = Z_near x joins the launch
    void up_and_translate_overlapped(int R, const cx<T> *x, cx<T> *y) {
        for (int l = f_; l >= 4; --l) upward_level(l, R);
        std::vector<UpPhiJob<T>> ph;
        std::vector<int64_t> n2;
        size_t sh = 8 * 2 * 64 * sizeof(cx<T>);
        {
            const int l = 3;
            std::vector<ThetaJob<T>> th;
            std::vector<int64_t> n1;
            size_t sh1 = 0;
            for (Reg &G : regs_) {
                const int nth_c = G.nth[l], nph_c = G.nph[l], nth_p = G.nth[l - 1], nph_p = G.nph[l - 1];
                th.push_back({G.nbox[l] * 2, nth_c, nph_c, nth_p, G.ipA[l], G.ipB[l], G.S[l], G.tmp});
                n1.push_back((int64_t)G.nbox[l] * 2 * ((nth_p + 1) / 2) * (nph_c / 2));
                sh1 = std::max(sh1, (size_t)2 * nth_p * nth_c * sizeof(T));
                ph.push_back({G.nbox[l - 1], nth_p, nph_p, nph_c, G.ipDt[l], G.child_ptr[l - 1], G.child_idx[l - 1],
                              G.slot[l], G.sup[l], G.tmp, G.S[l - 1]});
                n2.push_back((int64_t)G.nbox[l - 1] * 2 * nth_p * (nph_p / 2));
                sh = std::max(sh, (size_t)nph_c * nph_p * sizeof(T));
            }
            launch_jobs(th, n1, sh1, k_up_theta1<T, 64>, k_up_theta1<T, WG>);
        }
        JobList<UpPhiJob<T>> jl{};
        for (size_t i = 0; i < ph.size(); ++i) add_job(jl, ph[i], n2[i], WG);
        const TransGroups<T> tg = trans_groups(3, f_);
        const NearRows<T> none{};
        const unsigned grid = 8u * (unsigned)((jl.blk0[jl.n] + 7) / 8 + (tg.nblk + 7) / 8);
        if (grid) {
            k_near_up_phi1_translate1<T, false><<<grid, WG, sh, stream_>>>(jl, tg, none);
            LAUNCHCHK();
        }
        translate_level2_and_near(R, x, y);
    }
    // level 2: a few hundred workgroups; the near product's follow them
    void translate_level2_and_near(int R, const cx<T> *x, cx<T> *y) {
        const TransGroups<T> t2 = trans_groups(2, 2);
        if (x) {
            NearRows<T> nr{};
            nr.a = NearArgs<T>{R,  bstart_, near_col_ptr_, near_cols_, near_val_ptr_, nA_,    nB_,
                               nC_, x,       y,             nullptr,    cx<T>{0, 0},   1,      nullptr, nD_};
            nr.grp = near_grp_;
            nr.ngrp = near_ngrp_;
            const size_t sh2 = std::max((size_t)8 * 2 * 64 * sizeof(cx<T>), (size_t)max_ncol_ * 2 * sizeof(cx<T>));
            const unsigned g2 = 8u * (unsigned)((t2.nblk + 7) / 8 + (nr.ngrp + 7) / 8);
            if (gen_) k_near_up_phi1_translate1<T, true, true><<<g2, WG, sh2, stream_>>>(JobList<UpPhiJob<T>>{}, t2, nr);
            else k_near_up_phi1_translate1<T, true><<<g2, WG, sh2, stream_>>>(JobList<UpPhiJob<T>>{}, t2, nr);
            LAUNCHCHK();
        } else if (t2.nblk > 0) {
            k_translate_grp1<T><<<(unsigned)((t2.nblk + 7) / 8 * 8), WG, 0, stream_>>>(t2);
            LAUNCHCHK();
        }
    }

    // every translation level of every region; one RHS: one launch
    void translate_all(int R) {
        const int nlev = f_ - 1;
        if (R == 1 && nlev >= 1 && (int)regs_.size() * nlev <= TRANS_MAXJOB) {
            int nblk = 0;
            if (plan_.trans_grp) {
                const TransGroups<T> tg = trans_groups(2, f_);
                nblk = tg.nblk;
                if (nblk > 0) {
                    k_translate_grp1<T><<<(unsigned)((nblk + 7) / 8 * 8), WG, 0, stream_>>>(tg);
                    LAUNCHCHK();
                }
            } else {
                TransLevels<T> tl{};
                int e = 0;
                for (Reg &G : regs_)
                    for (int l = 2; l <= f_; ++l, ++e) {
                        tl.blk0[e] = nblk;
                        tl.K[e] = G.K[l];
                        tl.nkc[e] = (G.K[l] + 63) / 64;
                        tl.il_ptr[e] = G.il_ptr[l];
                        tl.il_src[e] = G.il_src[l];
                        tl.il_off[e] = G.il_off[l];
                        tl.trans[e] = G.trans[l];
                        tl.S[e] = G.S[l];
                        tl.G[e] = G.G[l];
                        nblk += G.nbox[l] * tl.nkc[e];
                    }
                tl.nlev = e;
                tl.blk0[e] = nblk;
                tl.nblk = nblk;
                if (nblk > 0) {
                    k_translate1<T><<<(unsigned)((nblk + 7) / 8 * 8), WG, 0, stream_>>>(tl);
                    LAUNCHCHK();
                }
            }
            return;
        }
        for (Reg &G : regs_)
            for (int l = 2; l <= f_; ++l) translate(G, l, R);
    }

    void translate(Reg &G, int l, int R) {
        if (!plan_.trans_grp) {
            k_translate<T><<<nblocks((int64_t)G.nbox[l] * G.K[l] * R), WG, 0, stream_>>>(
                G.nbox[l], G.K[l], R, G.il_ptr[l], G.il_src[l], G.il_off[l], G.trans[l], G.S[l], G.G[l]);
            LAUNCHCHK();
            return;
        }
        int rp = 1;
        while (rp < R) rp <<= 1;
        const int dpw = WG / rp;
        dim3 grid((G.ngrp[l] + 7) / 8 * 8, (G.K[l] + dpw - 1) / dpw);
#define SFMM_TG(RP_)                                                                                             \
    k_translate_grp<T, RP_><<<grid, WG, 0, stream_>>>(G.K[l], R, G.grp_dst[l], G.cand_ptr[l], G.cand_src[l], \
                                                      G.cand_off[l], G.trans[l], G.S[l], G.G[l],             \
                                                      G.ngrp[l])
        if (rp == 64) SFMM_TG(64);
        else if (rp == 32) SFMM_TG(32);
        else if (rp == 16) SFMM_TG(16);
        else if (rp == 8) SFMM_TG(8);
        else if (rp == 4) SFMM_TG(4);
        else if (rp == 2) SFMM_TG(2);
        else SFMM_TG(1);
#undef SFMM_TG
        LAUNCHCHK();
    }

    // Level transition l -> l - 1 (upward) or l - 1 -> l (downward) of every
    // region: one RHS with the split stages of all regions in one launch per
    // stage, otherwise region by region.
    template <typename P>
    static unsigned add_job(JobList<P> &jl, const P &p, int64_t items, int bs) {
        jl.blk0[jl.n] = jl.n ? jl.blk0[jl.n] : 0;
        jl.p[jl.n] = p;
        const unsigned nb = nblocks(items, bs);
        jl.blk0[jl.n + 1] = jl.blk0[jl.n] + (int)nb;
        ++jl.n;
        return nb;
    }
    bool split_all(int l, int R) const {
        if ((int)regs_.size() > SPLIT_MAXJOB) return false;
        for (const Reg &G : regs_) {
            if (!split_ok(G, l, R)) return false;
            // the kernels index their items in 32 bits
            const int64_t up = (int64_t)G.nbox[l] * 2 * G.nth[l - 1] * G.nph[l],
                          dn = (int64_t)std::max(G.nbox[l - 1], G.nbox[l]) * 2 * G.nth[l - 1] * G.nph[l - 1];
            if (std::max(up, dn) + 1024 >= ((int64_t)1 << 31)) return false;
        }
        return true;
    }
    template <typename P, typename K64, typename K256>
    void launch_jobs(const std::vector<P> &jobs, const std::vector<int64_t> &items, size_t shm, K64 k64,
                     K256 k256) {
        int64_t total = 0;
        for (int64_t n : items) total += n;
        const bool small = small_grid(total);
        const int bs = small ? 64 : WG;
        JobList<P> jl{};
        for (size_t i = 0; i < jobs.size(); ++i) add_job(jl, jobs[i], items[i], bs);
        const unsigned grid = (unsigned)jl.blk0[jl.n];
        if (!grid) return;
        if (small) k64<<<grid, 64, shm, stream_>>>(jl);
        else k256<<<grid, WG, shm, stream_>>>(jl);
        LAUNCHCHK();
    }
    void upward_level(int l, int R) {
        if (!split_all(l, R)) {
            for (Reg &G : regs_) upward(G, l, R);
            return;
        }
        std::vector<ThetaJob<T>> th;
        std::vector<UpPhiJob<T>> ph;
        std::vector<int64_t> n1, n2;
        size_t sh1 = 0, sh2 = 0;
        for (Reg &G : regs_) {
            const int nth_c = G.nth[l], nph_c = G.nph[l], nth_p = G.nth[l - 1], nph_p = G.nph[l - 1];
            th.push_back({G.nbox[l] * 2, nth_c, nph_c, nth_p, G.ipA[l], G.ipB[l], G.S[l], G.tmp});
            n1.push_back((int64_t)G.nbox[l] * 2 * ((nth_p + 1) / 2) * (nph_c / 2));
            sh1 = std::max(sh1, (size_t)2 * nth_p * nth_c * sizeof(T));
            ph.push_back({G.nbox[l - 1], nth_p, nph_p, nph_c, G.ipDt[l], G.child_ptr[l - 1], G.child_idx[l - 1],
                          G.slot[l], G.sup[l], G.tmp, G.S[l - 1]});
            n2.push_back((int64_t)G.nbox[l - 1] * 2 * nth_p * (nph_p / 2));
            sh2 = std::max(sh2, (size_t)nph_c * nph_p * sizeof(T));
        }
        launch_jobs(th, n1, sh1, k_up_theta1<T, 64>, k_up_theta1<T, WG>);
        launch_jobs(ph, n2, sh2, k_up_phi1<T, 64>, k_up_phi1<T, WG>);
    }
    void downward_level(int l, int R) {
        if (fused_ok(l, R)) {
            size_t sh = 0;
            const JobList<FusedDnJob<T>> jl = fused_dn_jobs(l, sh);
            if (jl.blk0[jl.n]) {
                k_dn_fused1<T><<<(unsigned)jl.blk0[jl.n], WG, sh, stream_>>>(jl);
                LAUNCHCHK();
            }
            return;
        }
        if (!split_all(l, R)) {
            for (Reg &G : regs_) downward(G, l, R);
            return;
        }
        std::vector<DnPhiJob<T>> ph;
        std::vector<ThetaJob<T>> th;
        std::vector<int64_t> n1, n2;
        size_t sh1 = 0, sh2 = 0;
        for (Reg &G : regs_) {
            const int nth_c = G.nth[l], nph_c = G.nph[l], nth_p = G.nth[l - 1], nph_p = G.nph[l - 1];
            ph.push_back({G.nbox[l], nth_p, nph_p, nph_c, G.ipD[l], G.parent[l], G.slot[l], G.sdn[l], G.G[l - 1],
                          G.tmp});
            n1.push_back((int64_t)G.nbox[l] * 2 * nth_p * (nph_c / 2));
            sh1 = std::max(sh1, (size_t)nph_p * nph_c * sizeof(T));
            th.push_back({G.nbox[l] * 2, nth_c, nph_c, nth_p, G.ipA[l], G.ipB[l], G.tmp, G.G[l]});
            n2.push_back((int64_t)G.nbox[l] * 2 * ((nth_c + 1) / 2) * (nph_c / 2));
            sh2 = std::max(sh2, (size_t)2 * nth_p * nth_c * sizeof(T));
        }
        launch_jobs(ph, n1, sh1, k_dn_phi1<T, 64>, k_dn_phi1<T, WG>);
        launch_jobs(th, n2, sh2, k_dn_theta1<T, 64>, k_dn_theta1<T, WG>);
    }

    void upward(Reg &G, int l, int R) {
        const int nth_c = G.nth[l], nph_c = G.nph[l], nth_p = G.nth[l - 1], nph_p = G.nph[l - 1];
        if constexpr (std::is_same<T, float>::value) {
            if (interp_mma_ok(G, l, R)) {
                upward_mma(G, l, R);
                return;
            }
        }
        const int rt = pick_tile(R, {4, 2, 1}, [&](int t) {
            return ((size_t)G.K[l] + (size_t)UPR * nph_c) * t * sizeof(cx<T>) <= LDS_LIMIT &&
                   UPR * nph_p * t <= WG * UPMAX;
        });
        if (rt) {
            const size_t shm = ((size_t)G.K[l] + (size_t)UPR * nph_c) * rt * sizeof(cx<T>);
            const int nchunk = (nth_p + UPR - 1) / UPR;
            const unsigned grid = (unsigned)G.nbox[l - 1] * 2 * nchunk * (R / rt);
#define SFMM_UP(RT_)                                                                                                 \
    k_up_box<T, RT_><<<grid, WG, shm, stream_>>>(R, nth_c, nph_c, nth_p, nph_p, G.ipA[l], G.ipB[l], G.ipDt[l],       \
                                                 G.child_ptr[l - 1], G.child_idx[l - 1], G.slot[l], G.sup[l], G.S[l], \
                                                 G.S[l - 1])
            if (rt == 4) SFMM_UP(4);
            else if (rt == 2) SFMM_UP(2);
            else SFMM_UP(1);
#undef SFMM_UP
            LAUNCHCHK();
            return;
        }
        const int64_t n1 = (int64_t)G.nbox[l] * 2 * nth_p * nph_c * R;
        k_up_theta<T><<<nblocks(n1), WG, 0, stream_>>>(R, G.nbox[l], nth_c, nph_c, nth_p, G.ipA[l], G.ipB[l], G.S[l],
                                                       G.tmp);
        LAUNCHCHK();
        const int64_t n2 = (int64_t)G.nbox[l - 1] * 2 * G.K[l - 1] * R;
        k_up_phi<T><<<nblocks(n2), WG, 0, stream_>>>(R, G.nbox[l - 1], nth_p, nph_p, nph_c, G.ipDt[l],
                                                     G.child_ptr[l - 1], G.child_idx[l - 1], G.slot[l], G.sup[l],
                                                     G.tmp, G.S[l - 1]);
        LAUNCHCHK();
    }

    void downward(Reg &G, int l, int R) {
        const int nth_c = G.nth[l], nph_c = G.nph[l], nth_p = G.nth[l - 1], nph_p = G.nph[l - 1];
        if constexpr (std::is_same<T, float>::value) {
            if (interp_mma_ok(G, l, R)) {
                downward_mma(G, l, R);
                return;
            }
        }
        const int rt = pick_tile(R, {4, 2, 1}, [&](int t) {
            return ((size_t)G.K[l - 1] + (size_t)nth_p * nph_c) * t * sizeof(cx<T>) <= LDS_LIMIT;
        });
        if (rt) {
            const size_t shm = ((size_t)G.K[l - 1] + (size_t)nth_p * nph_c) * rt * sizeof(cx<T>);
            const unsigned grid = (unsigned)G.nbox[l] * (R / rt);
#define SFMM_DN(RT_)                                                                                          \
    k_dn_box<T, RT_><<<grid, WG, shm, stream_>>>(R, nth_c, nph_c, nth_p, nph_p, G.ipA[l], G.ipB[l], G.ipD[l], \
                                                 G.parent[l], G.slot[l], G.sdn[l], G.G[l - 1], G.G[l])
            if (rt == 4) SFMM_DN(4);
            else if (rt == 2) SFMM_DN(2);
            else SFMM_DN(1);
#undef SFMM_DN
            LAUNCHCHK();
            return;
        }
        const int64_t n1 = (int64_t)G.nbox[l] * 2 * nth_p * nph_c * R;
        k_dn_phi<T><<<nblocks(n1), WG, 0, stream_>>>(R, G.nbox[l], nth_p, nph_p, nph_c, G.ipD[l], G.parent[l],
                                                     G.slot[l], G.sdn[l], G.G[l - 1], G.tmp);
        LAUNCHCHK();
        const int64_t n2 = (int64_t)G.nbox[l] * 2 * G.K[l] * R;
        k_dn_theta<T><<<nblocks(n2), WG, 0, stream_>>>(R, G.nbox[l], nth_c, nph_c, nth_p, G.ipA[l], G.ipB[l], G.tmp,
                                                       G.G[l]);
        LAUNCHCHK();
    }

    void ilu_sweep(int R, int box0, int n, const int *cp, const int *cl, const int64_t *vp, const cx<T> *W,
                   const cx<T> *own, const cx<T> *other, cx<T> *out) {
        if (!n) return;
        const int rt = pick_tile(R, {8, 4, 2, 1},
                                 [&](int t) { return (size_t)max_ilu_nc_ * 2 * t * sizeof(cx<T>) <= LDS_LIMIT; });
        const bool lds = rt > 0;
        const int t = lds ? rt : 1;
        dim3 grid(n, (2 * max_nrow_ + RW - 1) / RW, R / t);
        const size_t shm = lds ? (size_t)max_ilu_nc_ * 2 * t * sizeof(cx<T>) : 0;
#define SFMM_ILU(RT_, L_) \
    k_ilu<T, RT_, L_><<<grid, RWG, shm, stream_>>>(R, box0, bstart_, cp, cl, vp, W, own, other, out)
        if (!lds) SFMM_ILU(1, false);
        else if (t == 8) SFMM_ILU(8, true);
        else if (t == 4) SFMM_ILU(4, true);
        else if (t == 2) SFMM_ILU(2, true);
        else SFMM_ILU(1, true);
#undef SFMM_ILU
        LAUNCHCHK();
    }

    // w = M^-1 v for R right-hand sides (uses zi_ and pt_ as work space)
    void precond_internal(const cx<T> *v, cx<T> *w, int R) {
        const int64_t NR = (int64_t)2 * ne_ * R;
        if (profiling_) HIPCHK(hipEventRecord(ev0_, stream_));
        if (precond_ == SFMM_PRECOND_NONE) {
            HIPCHK(hipMemcpyAsync(w, v, sizeof(cx<T>) * NR, hipMemcpyDeviceToDevice, stream_));
        } else if (precond_ == SFMM_PRECOND_POLY) {
            k_zero<T><<<nblocks(NR), WG, 0, stream_>>>(w, NR);
            LAUNCHCHK();
            // p(D^-1 Z_near) D^-1 v in product form; every step's D^-1 is
            // applied in the near kernel's epilogue
            const cx<T> *cur = v;
            if (dinv_) {
                k_edge_block<T><<<nblocks((int64_t)ne_ * R), WG, 0, stream_>>>(ne_, R, dinv_, v, zi_);
                LAUNCHCHK();
                cur = zi_;
            }
            const int d = (int)inv_theta_.size();
            for (int k = 0; k < d; ++k) {
                cx<T> *next = (cur == zi_) ? pt_ : zi_;
                launch_near<true>(R, cur, next, w, inv_theta_[k], k < d - 1);
                cur = next;
            }
        } else if (precond_ == SFMM_PRECOND_BLOCK_JACOBI) {
            ilu_sweep(R, 0, nb_, fcol_ptr_, fcols_, fptr_, fval_, v, v, w);
        } else {
            for (int c = 0; c < 8; ++c)
                ilu_sweep(R, colour_ptr_[c], colour_ptr_[c + 1] - colour_ptr_[c], fcol_ptr_, fcols_, fptr_, fval_, v,
                          zi_, zi_);
            for (int c = 7; c >= 0; --c)
                ilu_sweep(R, colour_ptr_[c], colour_ptr_[c + 1] - colour_ptr_[c], bcol_ptr_, bcols_, bptr_, bval_, zi_,
                          w, w);
        }
        if (profiling_) {
            HIPCHK(hipEventRecord(ev1_, stream_));
            HIPCHK(hipEventSynchronize(ev1_));
            float ms = 0;
            HIPCHK(hipEventElapsedTime(&ms, ev0_, ev1_));
            times_.ms[6] += ms / R;
            times_.n[6] += 1;
        }
    }

    // ---- C ABI operations (boundary layout FP64 on device) ----
    void matvec(int n_rhs, const void *x_dev, void *y_dev, int parts) override {
        const int N = 2 * ne_;
        for (int r0 = 0; r0 < n_rhs; r0 += BATCH) {
            const int R = std::min(BATCH, n_rhs - r0);
            ensure_batch(R);
            use_plan(R);
            k_to_internal<T><<<nblocks((int64_t)ne_ * R), WG, 0, stream_>>>((const double2 *)x_dev + (size_t)r0 * N,
                                                                             pos_, ne_, R, xi_);
            LAUNCHCHK();
            if (parts == SFMM_PART_ALL) run_graph(G_PRODUCT, R, [&] { matvec_internal(xi_, yi_, R, parts); });
            else matvec_internal(xi_, yi_, R, parts);
            k_to_boundary<T><<<nblocks((int64_t)ne_ * R), WG, 0, stream_>>>(yi_, pos_, ne_, R,
                                                                             (double2 *)y_dev + (size_t)r0 * N);
            LAUNCHCHK();
        }
    }

    void precond(int n_rhs, const void *x_dev, void *y_dev) override {
        const int N = 2 * ne_;
        for (int r0 = 0; r0 < n_rhs; r0 += BATCH) {
            const int R = std::min(BATCH, n_rhs - r0);
            ensure_batch(R);
            use_plan(R);
            k_to_internal<T><<<nblocks((int64_t)ne_ * R), WG, 0, stream_>>>((const double2 *)x_dev + (size_t)r0 * N,
                                                                             pos_, ne_, R, xi_);
            LAUNCHCHK();
            run_graph(G_PRECOND, R, [&] { precond_internal(xi_, wi_, R); });
            k_to_boundary<T><<<nblocks((int64_t)ne_ * R), WG, 0, stream_>>>(wi_, pos_, ne_, R,
                                                                             (double2 *)y_dev + (size_t)r0 * N);
            LAUNCHCHK();
        }
    }

    // out[s] = A M^-1 in[s] (or A in[s], or M^-1 in[s]) for the Ra active
    // slots; zout[s] receives M^-1 in[s] exactly as the product saw it.
    void op_apply(const double2 *in, double2 *out, double2 *zout, int Ra, bool prec, bool prod) {
        const int N = 2 * ne_;
        const int64_t NR = (int64_t)N * Ra;
        use_plan(Ra);
        k_gather<T><<<nblocks(NR), WG, 0, stream_>>>(in, N, dact_, N, Ra, xi_);
        LAUNCHCHK();
        // the fixed-buffer part runs as one graph; the gathers and scatters
        // (whose vectors change every step) stay outside
        if (prec && prod) {
            run_graph(G_PREC_PRODUCT, Ra, [&] {
                precond_internal(xi_, wi_, Ra);
                matvec_internal(wi_, yi_, Ra, SFMM_PART_ALL);
            });
        } else if (prec) {
            run_graph(G_PRECOND, Ra, [&] { precond_internal(xi_, wi_, Ra); });
        } else if (prod) {
            run_graph(G_PRODUCT, Ra, [&] { matvec_internal(xi_, yi_, Ra, SFMM_PART_ALL); });
        }
        const cx<T> *z = prec ? wi_ : xi_;
        if (zout) {
            k_scatter<T><<<nblocks(NR), WG, 0, stream_>>>(z, N, Ra, dact_, N, zout);
            LAUNCHCHK();
        }
        k_scatter<T><<<nblocks(NR), WG, 0, stream_>>>(prod ? yi_ : z, N, Ra, dact_, N, out);
        LAUNCHCHK();
    }

    // 2-norms of the Ra active slot vectors at base
    std::vector<double> norms(const double2 *base, int Ra) {
        const int N = 2 * ne_;
        k_bnorm2<<<dim3(red_blocks_, Ra), WG, 0, stream_>>>(base, N, dact_, N, dpart_);
        LAUNCHCHK();
        k_sum_real<<<Ra, 64, 0, stream_>>>(dpart_, red_blocks_, dscal_);
        LAUNCHCHK();
        std::vector<double> s(Ra);
        copy_d2h(s.data(), dscal_, sizeof(double) * Ra, stream_);
        for (double &v : s) v = std::sqrt(v);
        return s;
    }

    void upload_act(const std::vector<int> &act) {
        stage_h2d(dact_, act.data(), sizeof(int) * act.size());
    }

    void solve(int solver, int n_rhs, const void *b_dev, void *x_dev, const void *x0_dev, int m, int max_iters,
               double tol, sfmm_solve_info *info, int verbose) override {
        if (solver == SFMM_SOLVER_GMRES) solve_gmres(n_rhs, b_dev, x_dev, x0_dev, m, max_iters, tol, info, verbose);
        else solve_bicg(solver == SFMM_SOLVER_CGS, n_rhs, b_dev, x_dev, x0_dev, max_iters, tol, info, verbose);
    }

    // out[a] = conj(X[act[a]]) . Y[act[a]] for the Ra active slots
    std::vector<cd> bdot(const double2 *X, const double2 *Y, int Ra) {
        const int N = 2 * ne_;
        k_bdots<<<dim3(red_blocks_, 1, Ra), WG, 0, stream_>>>(X, 0, N, Y, dact_, N, 1, dpartc_);
        LAUNCHCHK();
        k_sum_partials<<<Ra, 64, 0, stream_>>>(dpartc_, red_blocks_, dh_);
        LAUNCHCHK();
        std::vector<double2> h(Ra);
        copy_d2h(h.data(), dh_, sizeof(double2) * Ra, stream_);
        std::vector<cd> out(Ra);
        for (int a = 0; a < Ra; ++a) out[a] = cd(h[a].x, h[a].y);
        return out;
    }

    // out = c0 x + c1 y + c2 z per active slot (coefficients [Ra][3])
    void blin3(const std::vector<cd> &c, int Ra, const double2 *x, const double2 *y, const double2 *z,
               double2 *out) {
        const int N = 2 * ne_;
        std::vector<double2> cc(3 * (size_t)Ra);
        for (size_t i = 0; i < cc.size(); ++i) cc[i] = make_double2(c[i].real(), c[i].imag());
        stage_h2d(dh_, cc.data(), sizeof(double2) * cc.size());
        k_blin3<<<dim3(nblocks(N), Ra), WG, 0, stream_>>>(dh_, dact_, N, N, x, y, z, out);
        LAUNCHCHK();
    }

    // BiCGStab (van der Vorst 1992) or CGS (Sonneveld 1989), right
    // preconditioned (A M^-1 u = b, x = M^-1 u, the iterate x kept directly),
    // FP64 recurrences, right-hand sides in lockstep.  A right-hand side
    // leaves the batch when its explicitly recomputed residual reaches tol;
    // when the recurrence claims convergence but the true residual does not
    // confirm it, or an inner product vanishes, the right-hand side restarts
    // from its current iterate.
    void solve_bicg(bool cgs, int n_rhs, const void *b_dev, void *x_dev, const void *x0_dev, int max_iters,
                    double tol, sfmm_solve_info *info, int verbose) {
        const int N = 2 * ne_;
        bool all_ok = true;
        for (int c0 = 0; c0 < n_rhs; c0 += BATCH) {
            const int R = std::min(BATCH, n_rhs - c0);
            auto t0 = std::chrono::steady_clock::now();
            ensure_krylov(8, R);
            ensure_batch(R);
            const int64_t ldj = (int64_t)kR_ * N;
            double2 *r = kV_, *rh = kV_ + ldj, *p = kV_ + 2 * ldj, *v = kV_ + 3 * ldj, *sv = kV_ + 4 * ldj,
                    *tv = kV_ + 5 * ldj, *w = kV_ + 6 * ldj, *aw = kV_ + 7 * ldj;
            double2 *ph = kZ_, *sh = kZ_ + ldj;
            for (int s = 0; s < R; ++s) {
                k_perm_in<<<nblocks(ne_), WG, 0, stream_>>>((const double2 *)b_dev + (size_t)(c0 + s) * N, pos_, ne_,
                                                             kb_ + (size_t)s * N);
                LAUNCHCHK();
                if (x0_dev) {
                    k_perm_in<<<nblocks(ne_), WG, 0, stream_>>>((const double2 *)x0_dev + (size_t)(c0 + s) * N, pos_,
                                                                 ne_, kx_ + (size_t)s * N);
                    LAUNCHCHK();
                }
            }
            if (!x0_dev) HIPCHK(hipMemsetAsync(kx_, 0, sizeof(double2) * (size_t)R * N, stream_));
            std::vector<int> act(R);
            for (int s = 0; s < R; ++s) act[s] = s;
            upload_act(act);
            std::vector<double> nb = norms(kb_, R);
            for (int s = 0; s < R; ++s)
                if (!std::isfinite(nb[s]))
                    throw Error(SFMM_E_INVALID_ARG, "right-hand side " + std::to_string(c0 + s) + " is not finite");
            std::vector<int> its(R, 0), restarts(R, 0), used(R, 0);
            std::vector<double> rel(R, 1.0), rel0(R, 1.0);
            std::vector<char> conv(R, 0);
            // per-slot recurrence scalars
            std::vector<cd> rho_old(R, 1.0), alpha(R, 1.0), omega(R, 1.0);
            std::vector<char> fresh(R, 1);
            // true residual r = b - A x of the listed slots; returns their
            // relative norms and (re)starts their recurrences from it
            auto restart_from_true = [&](const std::vector<int> &slots, bool first) {
                upload_act(slots);
                const int Ra = (int)slots.size();
                if (first && !x0_dev) {
                    for (int s : slots)
                        HIPCHK(hipMemcpyAsync(r + (size_t)s * N, kb_ + (size_t)s * N, sizeof(double2) * N,
                                              hipMemcpyDeviceToDevice, stream_));
                } else {
                    op_apply(kx_, r, nullptr, Ra, false, true);
                    k_brsub<<<dim3(nblocks(N), Ra), WG, 0, stream_>>>(kb_, dact_, N, N, r);
                    LAUNCHCHK();
                }
                std::vector<double> nr = norms(r, Ra);
                for (int a = 0; a < Ra; ++a) {
                    const int s = slots[a];
                    HIPCHK(hipMemcpyAsync(rh + (size_t)s * N, r + (size_t)s * N, sizeof(double2) * N,
                                          hipMemcpyDeviceToDevice, stream_));
                    HIPCHK(hipMemsetAsync(p + (size_t)s * N, 0, sizeof(double2) * N, stream_));
                    HIPCHK(hipMemsetAsync(v + (size_t)s * N, 0, sizeof(double2) * N, stream_));
                    rho_old[s] = alpha[s] = omega[s] = 1.0;
                    fresh[s] = 1;
                }
                return nr;
            };
            {
                std::vector<double> nr = restart_from_true(act, true);
                for (int a = 0; a < R; ++a) {
                    const int s = act[a];
                    if (nb[s] == 0.0) {
                        conv[s] = 1;
                        rel[s] = 0.0;
                        continue;
                    }
                    rel[s] = nr[a] / nb[s];
                    if (x0_dev) {
                        rel0[s] = rel[s];
                        if (rel[s] < 1.0) used[s] = 1;
                    }
                }
                if (x0_dev) {
                    // the true residual judges a supplied guess: one no better
                    // than zero is dropped
                    std::vector<int> drop;
                    for (int s = 0; s < R; ++s)
                        if (!conv[s] && !used[s]) drop.push_back(s);
                    for (int s : drop) HIPCHK(hipMemsetAsync(kx_ + (size_t)s * N, 0, sizeof(double2) * N, stream_));
                    if (!drop.empty()) {
                        std::vector<double> nr2 = restart_from_true(drop, false);
                        for (size_t a = 0; a < drop.size(); ++a) rel[drop[a]] = nr2[a] / nb[drop[a]];
                    }
                }
                for (int s = 0; s < R; ++s)
                    if (!conv[s] && rel[s] <= tol) conv[s] = 1;
            }
            while (true) {
                act.clear();
                for (int s = 0; s < R; ++s)
                    if (!conv[s] && its[s] < max_iters) act.push_back(s);
                if (act.empty()) break;
                const int Ra = (int)act.size();
                upload_act(act);
                std::vector<cd> rho = bdot(rh, r, Ra);
                std::vector<cd> c(3 * (size_t)Ra);
                std::vector<int> broke;
                for (int a = 0; a < Ra; ++a) {
                    const int s = act[a];
                    if (std::abs(rho[a]) == 0.0) broke.push_back(s);
                }
                if (cgs) {
                    // u = r + beta q ; p = u + beta q + beta^2 p   (q in v, u in sv)
                    for (int a = 0; a < Ra; ++a) {
                        const int s = act[a];
                        const cd beta = fresh[s] ? cd(0.0) : rho[a] / rho_old[s];
                        c[3 * a] = 1.0;
                        c[3 * a + 1] = beta;
                        c[3 * a + 2] = 0.0;
                    }
                    blin3(c, Ra, r, v, nullptr, sv);
                    for (int a = 0; a < Ra; ++a) {
                        const int s = act[a];
                        const cd beta = fresh[s] ? cd(0.0) : rho[a] / rho_old[s];
                        c[3 * a] = 1.0;
                        c[3 * a + 1] = beta;
                        c[3 * a + 2] = beta * beta;
                    }
                    blin3(c, Ra, sv, v, p, p);
                } else {
                    // p = r + beta (p - omega v)
                    for (int a = 0; a < Ra; ++a) {
                        const int s = act[a];
                        const cd beta = fresh[s] ? cd(0.0) : (rho[a] / rho_old[s]) * (alpha[s] / omega[s]);
                        c[3 * a] = 1.0;
                        c[3 * a + 1] = beta;
                        c[3 * a + 2] = -beta * omega[s];
                    }
                    blin3(c, Ra, r, p, v, p);
                }
                // tv = A M^-1 p, ph = M^-1 p
                op_apply(p, tv, ph, Ra, precond_ != SFMM_PRECOND_NONE, true);
                std::vector<cd> sig = bdot(rh, tv, Ra);
                for (int a = 0; a < Ra; ++a) {
                    const int s = act[a];
                    alpha[s] = std::abs(sig[a]) > 0 ? rho[a] / sig[a] : cd(0.0);
                    if (!(std::abs(sig[a]) > 0) && std::find(broke.begin(), broke.end(), s) == broke.end())
                        broke.push_back(s);
                    c[3 * a] = 1.0;
                    c[3 * a + 1] = -alpha[s];
                    c[3 * a + 2] = 0.0;
                }
                if (cgs) {
                    // q = u - alpha A p^ ; w = u + q ; aw = A M^-1 w, sh = M^-1 w
                    blin3(c, Ra, sv, tv, nullptr, v);
                    for (int a = 0; a < Ra; ++a) {
                        c[3 * a] = 1.0;
                        c[3 * a + 1] = 1.0;
                    }
                    blin3(c, Ra, sv, v, nullptr, w);
                    op_apply(w, aw, sh, Ra, precond_ != SFMM_PRECOND_NONE, true);
                    // x += alpha u^ ; r -= alpha A u^
                    for (int a = 0; a < Ra; ++a) {
                        const int s = act[a];
                        c[3 * a] = 1.0;
                        c[3 * a + 1] = alpha[s];
                    }
                    blin3(c, Ra, kx_, sh, nullptr, kx_);
                    for (int a = 0; a < Ra; ++a) c[3 * a + 1] = -alpha[act[a]];
                    blin3(c, Ra, r, aw, nullptr, r);
                } else {
                    // s = r - alpha v ; t = A M^-1 s, sh = M^-1 s
                    std::swap(v, tv);   // v = A M^-1 p
                    blin3(c, Ra, r, v, nullptr, sv);
                    op_apply(sv, tv, sh, Ra, precond_ != SFMM_PRECOND_NONE, true);
                    std::vector<cd> ts = bdot(tv, sv, Ra);
                    std::vector<cd> tt = bdot(tv, tv, Ra);
                    for (int a = 0; a < Ra; ++a) {
                        const int s = act[a];
                        omega[s] = std::abs(tt[a]) > 0 ? ts[a] / tt[a] : cd(0.0);
                        if (!(std::abs(omega[s]) > 0) && std::find(broke.begin(), broke.end(), s) == broke.end())
                            broke.push_back(s);
                        c[3 * a] = 1.0;
                        c[3 * a + 1] = alpha[s];
                        c[3 * a + 2] = omega[s];
                    }
                    // x += alpha p^ + omega s^ ; r = s - omega t
                    blin3(c, Ra, kx_, ph, sh, kx_);
                    for (int a = 0; a < Ra; ++a) {
                        const int s = act[a];
                        c[3 * a + 1] = -omega[s];
                        c[3 * a + 2] = 0.0;
                    }
                    blin3(c, Ra, sv, tv, nullptr, r);
                }
                for (int a = 0; a < Ra; ++a) {
                    const int s = act[a];
                    rho_old[s] = rho[a];
                    fresh[s] = 0;
                    ++its[s];
                }
                std::vector<double> nr = norms(r, Ra);
                std::vector<int> check;
                for (int a = 0; a < Ra; ++a) {
                    const int s = act[a];
                    rel[s] = nr[a] / nb[s];
                    const bool bad = std::find(broke.begin(), broke.end(), s) != broke.end() || !std::isfinite(rel[s]);
                    if (rel[s] <= tol || bad || its[s] >= max_iters) check.push_back(s);
                }
                if (check.empty()) continue;
                // confirm on the true residual; restart the rest from their iterates
                std::vector<double> tr = restart_from_true(check, false);
                for (size_t q = 0; q < check.size(); ++q) {
                    const int s = check[q];
                    rel[s] = tr[q] / nb[s];
                    if (rel[s] <= tol) conv[s] = 1;
                    else if (its[s] < max_iters) ++restarts[s];
                    if (verbose >= 2)
                        std::fprintf(stderr, "sfmm %s: rhs %d its %d true residual %.3e\n", cgs ? "cgs" : "bicgstab",
                                     c0 + s, its[s], rel[s]);
                }
            }
            for (int s = 0; s < R; ++s) {
                k_perm_out<<<nblocks(ne_), WG, 0, stream_>>>(kx_ + (size_t)s * N, pos_, ne_,
                                                              (double2 *)x_dev + (size_t)(c0 + s) * N);
                LAUNCHCHK();
            }
            HIPCHK(hipStreamSynchronize(stream_));
            const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            for (int s = 0; s < R; ++s) {
                if (info) {
                    info[c0 + s].converged = conv[s] ? 1 : 0;
                    info[c0 + s].iterations = its[s];
                    info[c0 + s].restarts = restarts[s];
                    info[c0 + s].guess_used = used[s];
                    info[c0 + s].true_residual = rel[s];
                    info[c0 + s].initial_residual = rel0[s];
                    info[c0 + s].seconds = secs;
                }
                all_ok = all_ok && conv[s];
            }
        }
        if (!all_ok)
            throw Error(SFMM_E_NOT_CONVERGED, std::string(cgs ? "CGS" : "BiCGStab") +
                                                  " did not reach the tolerance within max_iters");
    }

    void solve_gmres(int n_rhs, const void *b_dev, void *x_dev, const void *x0_dev, int m, int max_iters, double tol,
                     sfmm_solve_info *info, int verbose) {
        const int N = 2 * ne_;
        bool all_ok = true;
        for (int c0 = 0; c0 < n_rhs; c0 += BATCH) {
            const int R = std::min(BATCH, n_rhs - c0);
            auto t0 = std::chrono::steady_clock::now();
            ensure_krylov(m, R);
            ensure_batch(R);
            const int64_t ldj = (int64_t)kR_ * N;   // stride between basis indices
            for (int s = 0; s < R; ++s) {
                k_perm_in<<<nblocks(ne_), WG, 0, stream_>>>((const double2 *)b_dev + (size_t)(c0 + s) * N, pos_, ne_,
                                                             kb_ + (size_t)s * N);
                LAUNCHCHK();
                if (x0_dev) {
                    k_perm_in<<<nblocks(ne_), WG, 0, stream_>>>((const double2 *)x0_dev + (size_t)(c0 + s) * N, pos_,
                                                                 ne_, kx_ + (size_t)s * N);
                    LAUNCHCHK();
                }
            }
            if (!x0_dev) HIPCHK(hipMemsetAsync(kx_, 0, sizeof(double2) * (size_t)R * N, stream_));
            std::vector<int> all(R);
            for (int s = 0; s < R; ++s) all[s] = s;
            upload_act(all);
            std::vector<double> nb = norms(kb_, R);
            for (int s = 0; s < R; ++s)
                if (!std::isfinite(nb[s]))
                    throw Error(SFMM_E_INVALID_ARG, "right-hand side " + std::to_string(c0 + s) + " is not finite");
            std::vector<int> its(R, 0), restarts(R, 0), used(R, 0);
            std::vector<double> rel(R, 0.0), rel0(R, 1.0);
            std::vector<char> conv(R, 0);
            for (int s = 0; s < R; ++s)
                if (nb[s] == 0.0) conv[s] = 1;
            bool first = true;
            const bool prec = precond_ != SFMM_PRECOND_NONE;
            while (true) {
                // true residuals of the slots still running
                std::vector<int> act;
                for (int s = 0; s < R; ++s)
                    if (!conv[s]) act.push_back(s);
                if (act.empty()) break;
                int Ra = (int)act.size();
                upload_act(act);
                double2 *V0 = kV_;
                if (first && !x0_dev) {
                    for (int s : act)
                        HIPCHK(hipMemcpyAsync(V0 + (size_t)s * N, kb_ + (size_t)s * N, sizeof(double2) * N,
                                              hipMemcpyDeviceToDevice, stream_));
                } else {
                    op_apply(kx_, V0, nullptr, Ra, false, true);
                    k_brsub<<<dim3(nblocks(N), Ra), WG, 0, stream_>>>(kb_, dact_, N, N, V0);
                    LAUNCHCHK();
                }
                const bool judge = first && x0_dev;
                first = false;
                std::vector<double> beta = norms(V0, Ra);
                if (judge) {
                    // the true residual judges a supplied guess: one that is no
                    // better than zero is dropped and the slot starts from zero
                    for (int a = 0; a < Ra; ++a) {
                        const int s = act[a];
                        rel0[s] = beta[a] / nb[s];
                        if (rel0[s] < 1.0) {
                            used[s] = 1;
                            continue;
                        }
                        HIPCHK(hipMemsetAsync(kx_ + (size_t)s * N, 0, sizeof(double2) * N, stream_));
                        HIPCHK(hipMemcpyAsync(V0 + (size_t)s * N, kb_ + (size_t)s * N, sizeof(double2) * N,
                                              hipMemcpyDeviceToDevice, stream_));
                        beta[a] = nb[s];
                    }
                }
                std::vector<int> next;
                for (int a = 0; a < Ra; ++a) {
                    const int s = act[a];
                    rel[s] = beta[a] / nb[s];
                    if (verbose >= 2)
                        std::fprintf(stderr, "sfmm gmres: rhs %d restart %d its %d true residual %.3e\n", c0 + s,
                                     restarts[s], its[s], rel[s]);
                    if (rel[s] <= tol) conv[s] = 1;
                    else if (its[s] < max_iters) next.push_back(a);
                }
                if (next.empty()) break;
                // compact to the slots that iterate in this cycle
                std::vector<int> act2;
                std::vector<double> inv_beta, g0;
                for (int a : next) {
                    act2.push_back(act[a]);
                    inv_beta.push_back(1.0 / beta[a]);
                    g0.push_back(beta[a]);
                }
                act = act2;
                Ra = (int)act.size();
                upload_act(act);
                stage_h2d(dscal_, inv_beta.data(), sizeof(double) * Ra);
                k_bscale<<<dim3(nblocks(N), Ra), WG, 0, stream_>>>(dscal_, dact_, N, N, V0);
                LAUNCHCHK();
                std::vector<cd> H((size_t)Ra * (m + 1) * m, 0.0), g((size_t)Ra * (m + 1), 0.0), sn((size_t)Ra * m);
                std::vector<double> cs((size_t)Ra * m);
                std::vector<int> cnt(Ra, 0);
                std::vector<char> done(Ra, 0);
                for (int a = 0; a < Ra; ++a) g[(size_t)a * (m + 1)] = g0[a];
                auto Hs = [&](int a, int i, int j) -> cd & { return H[((size_t)a * (m + 1) + i) * m + j]; };
                // positions of the cycle still iterating: a slot whose residual
                // estimate has met the tolerance leaves the batch at once (its
                // Arnoldi relation is complete at cnt steps), so the products
                // of the rest of the cycle run on the smaller batch
                std::vector<int> cur(Ra);
                for (int a = 0; a < Ra; ++a) cur[a] = a;
                for (int j = 0; j < m; ++j) {
                    double2 *Vj = kV_ + (size_t)j * ldj;
                    double2 *W = kV_ + (size_t)(j + 1) * ldj;
                    {
                        std::vector<int> nc;
                        for (int a : cur)
                            if (!done[a]) nc.push_back(a);
                        if (nc.size() != cur.size() || j == 0) {
                            cur = nc;
                            std::vector<int> sub;
                            for (int a : cur) sub.push_back(act[a]);
                            upload_act(sub);
                        }
                    }
                    const int Rc = (int)cur.size();
                    op_apply(Vj, W, kZ_ + (size_t)j * ldj, Rc, prec, true);
                    for (int a : cur) ++its[act[a]];
                    // classical Gram-Schmidt, twice; both passes' coefficients
                    // and the new vector's norm come back in one read-back
                    const size_t nh = (size_t)Rc * (j + 1);
                    for (int pass = 0; pass < 2; ++pass) {
                        k_bdots<<<dim3(red_blocks_, j + 1, Rc), WG, 0, stream_>>>(kV_, ldj, N, W, dact_, N, j + 1,
                                                                                  dpartc_);
                        LAUNCHCHK();
                        k_sum_partials<<<Rc * (j + 1), 64, 0, stream_>>>(dpartc_, red_blocks_, dh2_ + pass * nh);
                        LAUNCHCHK();
                        k_bsub<<<dim3(nblocks(N), Rc), WG, 0, stream_>>>(kV_, ldj, N, j + 1, dact_, N,
                                                                          dh2_ + pass * nh, W);
                        LAUNCHCHK();
                    }
                    k_bnorm2<<<dim3(red_blocks_, Rc), WG, 0, stream_>>>(W, N, dact_, N, dpart_);
                    LAUNCHCHK();
                    k_sum_real<<<Rc, 64, 0, stream_>>>(dpart_, red_blocks_, dscal_);
                    LAUNCHCHK();
                    std::vector<double2> hh(2 * nh);
                    std::vector<double> hn(Rc);
                    HIPCHK(hipMemcpyAsync(hh.data(), dh2_, sizeof(double2) * hh.size(), hipMemcpyDeviceToHost,
                                          stream_));
                    HIPCHK(hipMemcpyAsync(hn.data(), dscal_, sizeof(double) * Rc, hipMemcpyDeviceToHost, stream_));
                    HIPCHK(hipStreamSynchronize(stream_));
                    std::vector<cd> hsum(nh);
                    for (size_t q = 0; q < nh; ++q) hsum[q] = cd(hh[q].x + hh[nh + q].x, hh[q].y + hh[nh + q].y);
                    for (double &v : hn) v = std::sqrt(v);
                    std::vector<double> sc(Rc);
                    for (int q = 0; q < Rc; ++q) {
                        const int a = cur[q];
                        for (int i = 0; i <= j; ++i) Hs(a, i, j) = hsum[(size_t)q * (j + 1) + i];
                        Hs(a, j + 1, j) = hn[q];
                        const bool breakdown = !(hn[q] > 0);
                        sc[q] = breakdown ? 0.0 : 1.0 / hn[q];
                        for (int i = 0; i < j; ++i) {
                            const cd x1 = Hs(a, i, j), x2 = Hs(a, i + 1, j);
                            const double c = cs[(size_t)a * m + i];
                            const cd sv = sn[(size_t)a * m + i];
                            Hs(a, i, j) = c * x1 + sv * x2;
                            Hs(a, i + 1, j) = -std::conj(sv) * x1 + c * x2;
                        }
                        const cd x1 = Hs(a, j, j), x2 = Hs(a, j + 1, j);
                        const double n1 = std::abs(x1), n2 = std::abs(x2);
                        double c;
                        cd sv;
                        if (n2 == 0) {
                            c = 1;
                            sv = 0;
                        } else if (n1 == 0) {
                            c = 0;
                            sv = std::conj(x2) / n2;
                        } else {
                            const double rho = std::hypot(n1, n2);
                            c = n1 / rho;
                            sv = (x1 / n1) * std::conj(x2) / rho;
                        }
                        cs[(size_t)a * m + j] = c;
                        sn[(size_t)a * m + j] = sv;
                        Hs(a, j, j) = c * x1 + sv * x2;
                        Hs(a, j + 1, j) = 0;
                        cd &gj = g[(size_t)a * (m + 1) + j];
                        g[(size_t)a * (m + 1) + j + 1] = -std::conj(sv) * gj;
                        gj = c * gj;
                        cnt[a] = j + 1;
                        const double est = std::abs(g[(size_t)a * (m + 1) + j + 1]) / nb[act[a]];
                        if (est <= tol || its[act[a]] >= max_iters || breakdown) done[a] = 1;
                    }
                    stage_h2d(dscal_, sc.data(), sizeof(double) * Rc);
                    k_bscale<<<dim3(nblocks(N), Rc), WG, 0, stream_>>>(dscal_, dact_, N, N, W);
                    LAUNCHCHK();
                    if (std::all_of(done.begin(), done.end(), [](char d) { return d != 0; })) break;
                }
                upload_act(act);   // the update below covers every slot of the cycle
                // x += Z y with y = H^-1 g over each slot's own step count
                std::vector<double2> ys((size_t)Ra * m, make_double2(0, 0));
                for (int a = 0; a < Ra; ++a) {
                    const int n = cnt[a];
                    std::vector<cd> y(n);
                    for (int i = n - 1; i >= 0; --i) {
                        cd s = g[(size_t)a * (m + 1) + i];
                        for (int l = i + 1; l < n; ++l) s -= Hs(a, i, l) * y[l];
                        y[i] = s / Hs(a, i, i);
                    }
                    for (int i = 0; i < n; ++i) ys[(size_t)a * m + i] = make_double2(y[i].real(), y[i].imag());
                    ++restarts[act[a]];
                }
                stage_h2d(dh_, ys.data(), sizeof(double2) * ys.size());
                stage_h2d(dcnt_, cnt.data(), sizeof(int) * Ra);
                k_bupdate<<<dim3(nblocks(N), Ra), WG, 0, stream_>>>(kZ_, ldj, N, m, dcnt_, dact_, N, dh_, kx_);
                LAUNCHCHK();
            }
            for (int s = 0; s < R; ++s) {
                k_perm_out<<<nblocks(ne_), WG, 0, stream_>>>(kx_ + (size_t)s * N, pos_, ne_,
                                                              (double2 *)x_dev + (size_t)(c0 + s) * N);
                LAUNCHCHK();
            }
            HIPCHK(hipStreamSynchronize(stream_));
            const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            for (int s = 0; s < R; ++s) {
                if (info) {
                    info[c0 + s].converged = conv[s] ? 1 : 0;
                    info[c0 + s].iterations = its[s];
                    info[c0 + s].restarts = restarts[s];
                    info[c0 + s].guess_used = used[s];
                    info[c0 + s].true_residual = rel[s];
                    info[c0 + s].initial_residual = rel0[s];
                    info[c0 + s].seconds = secs;
                }
                all_ok = all_ok && conv[s];
            }
        }
        if (!all_ok) throw Error(SFMM_E_NOT_CONVERGED, "GMRES did not reach the tolerance within max_iters");
    }

    void planewave_rhs(int n_rhs, const double *angles, const double *pol, void *b_dev) override {
        double *da = (double *)device_alloc(sizeof(double) * 3 * n_rhs);
        try {
            HIPCHK(hipMemcpyAsync(da, angles, sizeof(double) * 2 * n_rhs, hipMemcpyHostToDevice, stream_));
            if (pol) HIPCHK(hipMemcpyAsync(da + 2 * n_rhs, pol, sizeof(double) * n_rhs, hipMemcpyHostToDevice, stream_));
            k_planewave_rhs<<<nblocks((int64_t)ne_ * n_rhs), WG, 0, stream_>>>(
                ne_, n_rhs, gs0_, gqr_, gqf_, gqn_, (double)tang_.x, h_.mesh.k0, 1.0 / ETA0, da,
                pol ? da + 2 * n_rhs : nullptr, (double2 *)b_dev);
            LAUNCHCHK();
            HIPCHK(hipStreamSynchronize(stream_));
        } catch (...) {
            device_free(da);
            throw;
        }
        device_free(da);
    }

    // far field through device staging buffers dd [2 n_dirs] and
    // ds [2 n_dirs n_rhs]; synchronous
    void rcs_staged(int n_rhs, const void *x_dev, int n_dirs, const double *tp, double *sigma, double *dd,
                    double *ds) {
        HIPCHK(hipMemcpyAsync(dd, tp, sizeof(double) * 2 * n_dirs, hipMemcpyHostToDevice, stream_));
        dim3 grid(n_dirs, (n_rhs + RCS_RT - 1) / RCS_RT);
        k_far_field<false><<<grid, 256, 0, stream_>>>(ne_, n_rhs, gs0_, gqr_, gqf_, h_.mesh.k0, ETA0, dd,
                                                      (const double2 *)x_dev, ds, n_dirs);
        LAUNCHCHK();
        HIPCHK(hipMemcpyAsync(sigma, ds, sizeof(double) * 2 * (size_t)n_dirs * n_rhs, hipMemcpyDeviceToHost,
                              stream_));
        HIPCHK(hipStreamSynchronize(stream_));
    }

    void far_pattern(int n_rhs, const void *x_dev, int n_dirs, const double *dirs_dev, double *F_dev) override {
        if (n_rhs < 1 || n_dirs < 1 || n_dirs > 65535) throw Error(SFMM_E_INVALID_ARG, "far pattern: bad sizes");
        for (int c0 = 0; c0 < n_rhs; c0 += 65535 * RCS_RT) {   // grid.y limit
            const int c = std::min(n_rhs - c0, 65535 * RCS_RT);
            dim3 grid(n_dirs, (c + RCS_RT - 1) / RCS_RT);
            k_far_field<true><<<grid, 256, 0, stream_>>>(ne_, c, gs0_, gqr_, gqf_, h_.mesh.k0, ETA0, dirs_dev,
                                                         (const double2 *)x_dev + (int64_t)c0 * 2 * ne_,
                                                         F_dev + (int64_t)c0 * n_dirs * 4, n_dirs);
            LAUNCHCHK();
        }
    }

    void rcs(int n_rhs, const void *x_dev, int n_dirs, const double *tp, double *sigma) override {
        double *dd = (double *)device_alloc(sizeof(double) * 2 * n_dirs);
        double *ds = (double *)device_alloc(sizeof(double) * 2 * (size_t)n_dirs * n_rhs);
        try {
            rcs_staged(n_rhs, x_dev, n_dirs, tp, sigma, dd, ds);
        } catch (...) {
            device_free(dd);
            device_free(ds);
            throw;
        }
        device_free(dd);
        device_free(ds);
    }

    void rcs_noalloc(int n_rhs, const void *x_dev, int n_dirs, const double *tp, double *sigma) override {
        const size_t need = (size_t)2 * n_dirs + (size_t)2 * n_dirs * n_rhs;
        if (need > SFMM_SCRATCH_DOUBLES)
            throw Error(SFMM_E_INVALID_ARG, "n_dirs * (2 + 2 n_rhs) = " + std::to_string(need) +
                                                " exceeds the scratch of " + std::to_string(SFMM_SCRATCH_DOUBLES) +
                                                " doubles");
        rcs_staged(n_rhs, x_dev, n_dirs, tp, sigma, scratch_, scratch_ + 2 * (size_t)n_dirs);
    }

    // quadrature geometry of every edge for the excitation and far-field kernels
    void upload_edge_quadrature(const Mesh &m) {
        const TriRule &q = tri_rule();
        const int ne = m.ne;
        std::vector<double> qr((size_t)14 * 3 * ne), qf(qr.size());
        // JMCFIE / CNF: n x (unsigned half) at the same points, weighted
        std::vector<double> qn(gen_ ? qr.size() : 0);
        std::vector<int> s0(ne);
        for (int e = 0; e < ne; ++e) {
            // the basis restricted to the exterior region: its two triangles
            // there (none if the edge does not touch the exterior)
            s0[e] = m.edge_region_sign(e, 0);
            int side = 0;
            for (int i = 0; i < m.nside[e] && s0[e]; ++i) {
                const int tri = m.etri[e][i], fv = m.efree[e][i];
                const int rs = m.tri_region_sign(tri, 0);
                if (!rs || side == 2) continue;
                const double coef = s0[e] * rs * m.ecoef[e][i] * m.len[e] / (2.0 * m.area[tri]);
                for (int a = 0; a < 7; ++a) {
                    const V3 &r = m.qp[tri][a];
                    const double w = q.w[a] * m.area[tri];
                    const int qi = side * 7 + a;
                    for (int c = 0; c < 3; ++c) {
                        qr[((size_t)qi * 3 + c) * ne + e] = r[c];
                        qf[((size_t)qi * 3 + c) * ne + e] = coef * (r[c] - m.V[fv][c]) * w;
                    }
                    if (gen_) {
                        const double cu = m.ecoef[e][i] * m.len[e] / (2.0 * m.area[tri]) * w;
                        const V3 h = m.qp[tri][a] - m.V[fv];
                        const V3 &n = m.normal[tri];
                        const double nh[3] = {n[1] * h[2] - n[2] * h[1], n[2] * h[0] - n[0] * h[2],
                                              n[0] * h[1] - n[1] * h[0]};
                        for (int c = 0; c < 3; ++c) qn[((size_t)qi * 3 + c) * ne + e] = cu * nh[c];
                    }
                }
                ++side;
            }
        }
        gs0_ = upload(s0);
        gqr_ = upload(qr);
        gqf_ = upload(qf);
        if (gen_) gqn_ = upload(qn);
    }

  private:
    struct Reg {
        cx<T> et{}, inv_et{};
        bool lossy = false;
        int nbf = 0, max_ebox = 0;
        int *edge_ptr = nullptr, *edge_pos = nullptr, *edge_sign = nullptr;
        int *edge_box = nullptr;   // region box of every entry of the region's edge list
        int ne = 0;                // entries of the region's edge list
        cx<T> *tx = nullptr, *rx = nullptr, *tmp = nullptr;
        cx<T> *nx = nullptr;       // patterns of the rotated test functions (JMCFIE / CNF)
        int K[MAXLEV] = {0}, nth[MAXLEV] = {0}, nph[MAXLEV] = {0}, nbox[MAXLEV] = {0};
        cx<T> *S[MAXLEV] = {nullptr}, *G[MAXLEV] = {nullptr}, *trans[MAXLEV] = {nullptr};
        int *il_ptr[MAXLEV] = {nullptr}, *il_src[MAXLEV] = {nullptr}, *il_off[MAXLEV] = {nullptr};
        // translation groups (siblings of one parent): dst[g][octant], candidate sources, offsets
        int ngrp[MAXLEV] = {0};
        int *grp_dst[MAXLEV] = {nullptr}, *cand_ptr[MAXLEV] = {nullptr}, *cand_src[MAXLEV] = {nullptr};
        int *cand_off[MAXLEV] = {nullptr};
        int *parent[MAXLEV] = {nullptr}, *slot[MAXLEV] = {nullptr};
        int *child_ptr[MAXLEV] = {nullptr}, *child_idx[MAXLEV] = {nullptr};
        T *ipA[MAXLEV] = {nullptr}, *ipB[MAXLEV] = {nullptr}, *ipD[MAXLEV] = {nullptr}, *ipDt[MAXLEV] = {nullptr};
        cx<T> *sup[MAXLEV] = {nullptr}, *sdn[MAXLEV] = {nullptr};
        cx<T> *Dup[MAXLEV] = {nullptr}, *Ddn[MAXLEV] = {nullptr};   // shift-folded phi stages
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
    // (re, im) rounded to bfloat16 (to nearest even, through FP32), packed
    // low/high in 32 bits
    uint32_t *upload_bf16x2(const std::vector<cd> &v) {
        auto bf = [](double d) -> uint32_t {
            const float f = (float)d;
            uint32_t u;
            std::memcpy(&u, &f, 4);
            if ((u & 0x7f800000u) == 0x7f800000u) return u >> 16;   // inf / nan kept
            u += 0x7fffu + ((u >> 16) & 1u);
            return u >> 16;
        };
        std::vector<uint32_t> t(v.size());
        for (size_t i = 0; i < v.size(); ++i) t[i] = bf(v[i].real()) | (bf(v[i].imag()) << 16);
        return upload(t);
    }
    T *upload_real(const std::vector<double> &v) {
        std::vector<T> t(v.begin(), v.end());
        return upload(t);
    }
    template <typename U>
    U *alloc_in(std::vector<void *> &pool, size_t n) {
        U *p = (U *)device_alloc(sizeof(U) * std::max<size_t>(n, 1));
        pool.push_back(p);
        return p;
    }

    // vectors and level arrays for R right-hand sides
    void ensure_batch(int R) {
        if (R <= rcap_) return;
        HIPCHK(hipStreamSynchronize(stream_));
        clear_graphs();   // they hold the old buffer addresses
        for (void *p : batch_allocs_) device_free(p);
        batch_allocs_.clear();
        const size_t NR = (size_t)2 * ne_ * R;
        xi_ = alloc_in<cx<T>>(batch_allocs_, NR);
        yi_ = alloc_in<cx<T>>(batch_allocs_, NR);
        zi_ = alloc_in<cx<T>>(batch_allocs_, NR);
        wi_ = alloc_in<cx<T>>(batch_allocs_, NR);
        pt_ = alloc_in<cx<T>>(batch_allocs_, NR);
        for (Reg &G : regs_) {
            if (f_ < 2) continue;
            size_t tmp = 0;
            for (int l = 2; l <= f_; ++l) {
                G.S[l] = alloc_in<cx<T>>(batch_allocs_, (size_t)G.nbox[l] * 2 * G.K[l] * R);
                G.G[l] = alloc_in<cx<T>>(batch_allocs_, (size_t)G.nbox[l] * 2 * G.K[l] * R);
                if (l >= 3) tmp = std::max(tmp, (size_t)G.nbox[l] * 2 * G.nth[l - 1] * G.nph[l] * R);
            }
            G.tmp = tmp ? alloc_in<cx<T>>(batch_allocs_, tmp) : nullptr;
        }
        rcap_ = R;
    }

    void ensure_krylov(int m, int R) {
        const int N = 2 * ne_;
        if (m <= kM_ && R <= kR_) return;
        HIPCHK(hipStreamSynchronize(stream_));
        for (void *p : krylov_allocs_) device_free(p);
        krylov_allocs_.clear();
        kM_ = std::max(m, kM_);
        kR_ = std::max(R, kR_);
        kV_ = alloc_in<double2>(krylov_allocs_, (size_t)(kM_ + 1) * kR_ * N);
        kZ_ = alloc_in<double2>(krylov_allocs_, (size_t)kM_ * kR_ * N);
        kb_ = alloc_in<double2>(krylov_allocs_, (size_t)kR_ * N);
        kx_ = alloc_in<double2>(krylov_allocs_, (size_t)kR_ * N);
        red_blocks_ = std::min(128, (int)nblocks(N, WG * 4));
        dpartc_ = alloc_in<double2>(krylov_allocs_, (size_t)(kM_ + 1) * kR_ * red_blocks_);
        dpart_ = alloc_in<double>(krylov_allocs_, (size_t)kR_ * red_blocks_);
        dh_ = alloc_in<double2>(krylov_allocs_, (size_t)(kM_ + 1) * kR_);
        dh2_ = alloc_in<double2>(krylov_allocs_, (size_t)2 * (kM_ + 1) * kR_);
        dscal_ = alloc_in<double>(krylov_allocs_, kR_);
        dact_ = alloc_in<int>(krylov_allocs_, kR_);
        dcnt_ = alloc_in<int>(krylov_allocs_, kR_);
    }

    void mark(int i) {
        if (profiling_) HIPCHK(hipEventRecord(evs_[i], stream_));
    }
    void collect_matvec(int R) {
        HIPCHK(hipEventSynchronize(evs_[6]));
        float ms;
        for (int i = 0; i < 6; ++i) {
            HIPCHK(hipEventElapsedTime(&ms, evs_[i], evs_[i + 1]));
            times_.ms[i] += ms / R;
            times_.n[i] += 1;
        }
        HIPCHK(hipEventElapsedTime(&ms, evs_[0], evs_[6]));
        times_.ms[7] += ms / R;
        times_.n[7] += 1;
    }

    const BodyHost &h_;
    hipStream_t stream_;
    Rcv1All<T> rcv_all_{};   // single-RHS receive of all regions in one launch
    int ne_ = 0, nb_ = 0, f_ = 0;
    std::array<int, 9> colour_ptr_{};
    int *pos_ = nullptr, *bstart_ = nullptr;
    int *near_col_ptr_ = nullptr, *near_cols_ = nullptr;
    int64_t *near_val_ptr_ = nullptr;
    cx<T> *nA_ = nullptr, *nB_ = nullptr, *nC_ = nullptr;
    uint32_t *h16A_ = nullptr, *h16B_ = nullptr, *h16C_ = nullptr, *h16D_ = nullptr;
    // bfloat16 tiles of the polynomial preconditioner (build_poly_tiles)
    int pntiles_ = 0;
    int64_t pnsteps_ = 0;
    int *ptile_box_ = nullptr, *ptile_row0_ = nullptr;
    int64_t *ptile_step_ = nullptr;
    uint16_t *ptvals_ = nullptr;
    cx<T> *nD_ = nullptr;          // H-row J coefficient of the general block (JMCFIE / CNF)
    char *pin_ = nullptr;          // pinned staging arena of stage_h2d
    size_t pin_cap_ = 0, pin_off_ = 0;
    bool gen_ = false;             // JMCFIE or CNF: general near blocks, rotated-test receive
    cx<T> tang_{-1, 0};            // weight of the tangential parts (-1 JMCFIE, 0 CNF)
    // matrix-core tiles of the near matrix (FP32 / bf16-split modes)
    bool split_ = false;
    bool graphs_ = true;
    bool autotune_ = false;
    int kernel_plan_ = 0;
    int verbose_ = 0;
    Plan plan_{};
    std::map<int, Plan> plans_;
    hipStream_t own_stream_ = nullptr;
    std::map<std::pair<int, int>, hipGraphExec_t> gexec_;
    int ntiles_ = 0;
    int64_t nsteps_ = 0;
    int *tile_box_ = nullptr, *tile_row0_ = nullptr;
    int64_t *tile_step_ = nullptr;
    void *tvals_ = nullptr;
    // edge quadrature for the plane-wave and far-field kernels
    double *scratch_ = nullptr;   // this device's copy of `scratch`
    int *gs0_ = nullptr;
    double *gqr_ = nullptr, *gqf_ = nullptr, *gqn_ = nullptr;
    int *near_grp_ = nullptr, near_ngrp_ = 0;
    int max_ncol_ = 0, max_nrow_ = 0, max_ilu_nc_ = 0, precond_ = SFMM_PRECOND_ILU0;
    int *fcol_ptr_ = nullptr, *fcols_ = nullptr, *bcol_ptr_ = nullptr, *bcols_ = nullptr;
    int64_t *fptr_ = nullptr, *bptr_ = nullptr;
    cx<T> *fval_ = nullptr, *bval_ = nullptr;
    std::vector<cx<T>> inv_theta_;
    cx<T> *dinv_ = nullptr;   // edge-block scaling of the polynomial preconditioner
    std::vector<Reg> regs_;
    int rcap_ = 0;
    cx<T> *xi_ = nullptr, *yi_ = nullptr, *zi_ = nullptr, *wi_ = nullptr, *pt_ = nullptr;
    int kM_ = 0, kR_ = 0, red_blocks_ = 1;
    double2 *kV_ = nullptr, *kZ_ = nullptr, *kb_ = nullptr, *kx_ = nullptr;
    double2 *dpartc_ = nullptr, *dh_ = nullptr, *dh2_ = nullptr;
    double *dpart_ = nullptr, *dscal_ = nullptr;
    int *dact_ = nullptr, *dcnt_ = nullptr;
    std::vector<void *> allocs_, batch_allocs_, krylov_allocs_;
    int64_t bytes_ = 0;
    bool profiling_ = false;
    hipEvent_t ev0_ = nullptr, ev1_ = nullptr;
    hipEvent_t evs_[7] = {nullptr};
    StageTimes times_;
};

}  // namespace

std::unique_ptr<DeviceBody> make_device_body(const BodyHost &h, int precision, int device, void *stream,
                                             bool graphs, bool autotune, int kernel_plan, int verbose) {
    check_device(device);
    if (precision == SFMM_PREC_FP64)
        return std::make_unique<DeviceBodyT<double>>(h, device, stream, false, graphs, autotune, kernel_plan, verbose);
    if (precision == SFMM_PREC_FP32)
        return std::make_unique<DeviceBodyT<float>>(h, device, stream, false, graphs, autotune, kernel_plan, verbose);
    if (precision == SFMM_PREC_BF16_SPLIT)
        return std::make_unique<DeviceBodyT<float>>(h, device, stream, true, graphs, autotune, kernel_plan, verbose);
    throw Error(SFMM_E_UNSUPPORTED, "unknown precision mode");
}

}  // namespace sfmm
