"""Benchmark of the MLFMM-accelerated PMCHWT product on one MI355X.

Workload (the metric's single-GPU configuration): homogeneous dielectric
sphere, radius 2 wavelengths, eps_r = 2.56, icosphere subdivision 5 (20,480
triangles, 30,720 RWG edges, 61,440 unknowns), 5-level octree with
0.25-wavelength finest boxes, excess-bandwidth truncation for 3 digits,
complex FP32 products, one right-hand side.  Inputs are seeded
and synthetic (complex Gaussian vector, numpy default_rng(1234)) and resident
in HBM before timing starts.

A timed step is one MLFMM product y = Z x (near-field box-ELL product plus
aggregation, interpolation, translation, anterpolation and receive for both
regions) through the C ABI on device pointers.  value = unknowns x RHS per
second over the K timed steps.  The same run also reports, outside the timed
region: per-stage GPU times from HIP events on the library's stream, the
preconditioner time, GMRES(50) time-to-1e-4 for the x-polarised plane wave
along -z with the near-field polynomial preconditioner (with the iteration
count), the roofline of the whole product (the replayed graph of one product
is the unit: its algorithmic bytes over its HIP-event time), matrix-core
utilisation of the 64-RHS products, the 64-angle sweeps on the sphere and on
the 307,200-unknown two-layer coated sphere, and the CPU oracle on bounded
row samples (all host cores and one core).
"""

import argparse
import glob
import hashlib
import json
import multiprocessing
import os
import platform
import re
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "MLFMM matvec unknowns×RHS/s + GMRES time-to-1e-4 per angle vs plain GPU path"
HBM_PEAK_GBS = 8000.0
MFMA_PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2500.0}   # dense, MI355X
# HBM traffic of one replayed product, from two rocprofv3 --pmc runs of
# `bench.py --product-only` (FETCH_SIZE, WRITE_SIZE over every dispatch of the
# timed products, scaled by a plain device copy); the summary records a hash
# of the kernel sources it was taken with, and the figure is reported only
# while the sources still hash the same
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "mlfmm_product_sphere61440_fp32_pmc_traffic.md")


def kernel_sources_hash():
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_1704_06862_amd", "csrc", "*.hip")) +
                    glob.glob(os.path.join(ROOT, "paper_1704_06862_amd", "csrc", "*.hpp"))):
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """(bytes per product, note) from the committed counter summary, or
    (None, reason) when it is missing or the kernels changed since."""
    try:
        text = open(TRAFFIC_PROFILE).read()
    except OSError:
        return None, "no counter summary"
    b = re.search(r"traffic_bytes_per_product:\s*(\d+)", text)
    h = re.search(r"kernel_sources_sha256_16:\s*([0-9a-f]+)", text)
    if not b or not h:
        return None, "counter summary unreadable"
    if h.group(1) != kernel_sources_hash():
        return None, "kernels changed since the counters were taken"
    return int(b.group(1)), os.path.relpath(TRAFFIC_PROFILE, ROOT)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=50)
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-solve", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=15.0)
    p.add_argument("--batch", type=str, default="8,64",
                   help="extra right-hand-side batch sizes measured outside the timed region")
    p.add_argument("--sweep", type=int, default=64, help="angles of the theta sweep (0 = skip)")
    p.add_argument("--train-every", type=int, default=2,
                   help="learned-guess sweep: solve every n-th angle first and train on those")
    p.add_argument("--copy-calibration", type=int, default=0,
                   help="MiB of a plain device copy run after the measurements, to scale HBM byte counters")
    p.add_argument("--product-only", action="store_true",
                   help="only the timed single-RHS products (for counter runs)")
    p.add_argument("--product-rhs", type=int, default=1,
                   help="with --product-only: right-hand sides per timed product (1-64; counter runs of "
                        "the batched kernels)")
    p.add_argument("--no-graphs", action="store_true",
                   help="launch the products kernel by kernel instead of replaying captured graphs")
    p.add_argument("--no-coated", action="store_true",
                   help="skip the 307,200-unknown coated-sphere leg (64-RHS products and 64-angle sweep)")
    p.add_argument("--coated-plain-stride", type=int, default=8,
                   help="coated sweep: the plain single-RHS path is timed on every n-th angle")
    p.add_argument("--cylinder-sweep", type=int, default=0,
                   help="angles of the stacked-cylinder monostatic sweep under JMCFIE (0 = skip; 721 is the "
                        "three-layer workload's sweep)")
    p.add_argument("--cylinder-train-every", type=int, default=10,
                   help="stacked-cylinder sweep: the learned guess trains on every n-th angle")
    p.add_argument("--cylinder-plain-stride", type=int, default=8,
                   help="stacked-cylinder sweep: the plain single-RHS path is timed on every n-th angle")
    return p.parse_args()


def _oracle_rows(args):
    body, edges, x = args
    from threadpoolctl import threadpool_limits

    from oracle import mom, rwg

    mesh = rwg.from_body(body)
    with threadpool_limits(limits=1):
        ZE, ZH = mom.pmchwt_rows(mesh, body.eps_r, body.mu_r, body.frequency, edges)
        _ = ZE @ x, ZH @ x
    return len(edges)


def _cpu_model():
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        m = re.search(r"Model name:\s*(.+)", out)
        if m:
            return m.group(1).strip()
    except (OSError, subprocess.SubprocessError):
        pass
    return platform.processor() or "unknown"


def cpu_baseline(body, x, seconds):
    """The oracle computing sampled rows of Z x (E and H rows of seeded
    edges): on every host core (one process per core, one thread each) and on
    one core, ~seconds each.  A full product needs 2E rows, so rows per
    second = unknowns x RHS per second."""
    from oracle import rwg

    ne = rwg.from_body(body).n_edges
    order = np.random.default_rng(0).permutation(ne)
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    out = {}
    for label, procs in (("all", cores), ("one", 1)):
        done = 0
        t0 = time.perf_counter()
        ctx = multiprocessing.get_context("fork")
        with ctx.Pool(procs) as pool:
            while time.perf_counter() - t0 < seconds and done < ne:
                chunk = [(body, order[done + 2 * i: done + 2 * i + 2], x) for i in range(procs)]
                done += sum(pool.map(_oracle_rows, chunk))
        dt = time.perf_counter() - t0
        out[label] = (2 * done, dt, procs)
    rows, dt, procs = out["all"]
    rows1, dt1, _ = out["one"]
    return {"value": rows / dt, "unit": "unknowns*RHS/s", "cores": procs, "kind": "oracle",
            "sample": f"{rows} of {2 * ne} rows of Z x (dense PMCHWT rows with singular extraction, FP64 numpy) "
                      f"in {dt:.1f} s on {procs} processes of one thread",
            "cpu_model": _cpu_model(), "nproc": os.cpu_count(),
            "single_core": {"value": rows1 / dt1, "cores": 1,
                            "sample": f"{rows1} rows in {dt1:.1f} s on one process of one thread"}}


def sweep(ctx, ctx_mixed, torch, n_ang, every, plain_stride=1, batched_fp32=True, pretrained=True):
    """Time-to-solution of a theta sweep (theta uniform in [0, 180] degrees at
    phi = 0, theta-polarised) to the 1e-4 true residual:
      plain            FP32, one right-hand side per solve, zero start;
      batched          FP32, all angles in one lockstep solve;
      mixed            bf16-split matrix-core products, all angles at once;
      learned_in_sweep bf16-split: every `every`-th angle solved first (to
                       the tolerance: those angles are done), the network
                       trained on their currents, then the other angles
                       solved from its predictions (solves, training and
                       prediction all timed);
      learned_pretrained bf16-split, network trained beforehand on a coarse
                       sweep at the mid-points (reported apart): prediction and
                       one batched solve of all angles from it are timed;
      span_projection  the same training solutions without the network: the
                       minimal-residual guess in their POD span (baseline).
    """
    from workloads import theta_sweep

    n = ctx.sfmm_num_unknowns()
    ang = theta_sweep(n_ang)
    b = torch.zeros((n_ang, n), dtype=torch.complex128, device="cuda")
    ctx.sfmm_planewave_rhs(ang, b)
    torch.cuda.synchronize()

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        return out, time.perf_counter() - t0

    def its(infos):
        # mean and, since a batch iterates in lockstep, the maximum
        return [round(float(np.mean([i["iterations"] for i in infos])), 1), max(i["iterations"] for i in infos)]

    def plain_one(i):
        if i % 16 == 0:
            print(f"sweep: plain single-RHS solve {i} of {n_ang}", file=sys.stderr, flush=True)
        return ctx.sfmm_solve(b[i:i + 1], x[i:i + 1])[0]

    x = torch.zeros_like(b)
    plain_idx = list(range(0, n_ang, plain_stride))
    i_plain, t_plain = timed(lambda: [plain_one(i) for i in plain_idx])
    t_plain *= n_ang / len(plain_idx)           # per-angle rate of the subset, over the whole sweep
    print("sweep: batched solves", file=sys.stderr, flush=True)
    i_batch, t_batch = [], None
    if batched_fp32:
        x.zero_()
        i_batch, t_batch = timed(lambda: ctx.sfmm_solve(b, x))
    x.zero_()
    i_mixed, t_mixed = timed(lambda: ctx_mixed.sfmm_solve(b, x))

    tr = np.union1d(np.arange(0, n_ang, every), [n_ang - 1])   # both ends of the sweep: no extrapolation
    te = np.setdiff1d(np.arange(n_ang), tr)
    tr_t = torch.from_numpy(tr).to("cuda")
    te_t = torch.from_numpy(te).to("cuda")

    def learned():
        # the training angles are solved to the tolerance (they are then
        # done); the network learns their currents and starts the others
        b_tr = b.index_select(0, tr_t).contiguous()
        x_tr = torch.zeros_like(b_tr)
        i_tr = ctx_mixed.sfmm_solve(b_tr, x_tr)
        t_fit = time.perf_counter()
        loss = ctx_mixed.sfmm_guess_fit(ang[tr], x_tr)
        b_te = b.index_select(0, te_t).contiguous()
        x0 = torch.zeros_like(b_te)
        ctx_mixed.sfmm_guess_predict(ang[te], x0)
        torch.cuda.synchronize()
        t_fit = time.perf_counter() - t_fit
        x_te = torch.zeros_like(b_te)
        i_te = ctx_mixed.sfmm_solve(b_te, x_te, x0=x0)
        return i_tr, i_te, loss, t_fit, x_tr

    def span_in_sweep(x_tr):
        # the same protocol without the network: POD basis of the training
        # solutions (fit with no Adam steps), minimal-residual guess in its span
        parts = {}
        _, parts["fit_s"] = timed(lambda: ctx_mixed.sfmm_guess_fit(ang[tr], x_tr, epochs=0))
        b_te = b.index_select(0, te_t).contiguous()
        x0 = torch.zeros_like(b_te)
        _, parts["span_guess_s"] = timed(lambda: ctx_mixed.sfmm_span_predict(ang[te], x0))
        x_te = torch.zeros_like(b_te)
        info, parts["solve_s"] = timed(lambda: ctx_mixed.sfmm_solve(b_te, x_te, x0=x0))
        return info, {k: round(v, 3) for k, v in parts.items()}

    # a network trained beforehand on a coarse sweep (the mid-points of this
    # sweep's angles, every other one): prediction + one batched solve of all
    # angles is timed; the coarse solves and the training are reported apart
    mid = np.stack([np.deg2rad(np.linspace(0.0, 180.0, n_ang))[:-1:2] + np.deg2rad(90.0 / (n_ang - 1)),
                    np.zeros((n_ang - 1 + 1) // 2)], axis=1)
    b_mid = torch.zeros((len(mid), n), dtype=torch.complex128, device="cuda")
    ctx_mixed.sfmm_planewave_rhs(mid, b_mid)
    x_mid = torch.zeros_like(b_mid)

    def pretrain():
        i_mid = ctx_mixed.sfmm_solve(b_mid, x_mid)
        loss = ctx_mixed.sfmm_guess_fit(mid, x_mid)
        return i_mid, loss

    i_mid, i_am, i_sp = [], [], []
    if pretrained:
        (i_mid, loss_pre), t_pre = timed(pretrain)

        def amortized():
            x0 = torch.zeros_like(b)
            ctx_mixed.sfmm_guess_predict(ang, x0)
            xs = torch.zeros_like(b)
            return ctx_mixed.sfmm_solve(b, xs, x0=x0)

        i_am, t_am = timed(amortized)

        def span_baseline():
            x0 = torch.zeros_like(b)
            ctx_mixed.sfmm_span_predict(ang, x0)
            xs = torch.zeros_like(b)
            return ctx_mixed.sfmm_solve(b, xs, x0=x0)

        span_baseline()   # the first call forms Z U (reported with the training cost)
        i_sp, t_sp = timed(span_baseline)

    print("sweep: learned guess inside the sweep", file=sys.stderr, flush=True)
    (i_tr, i_te, loss, t_fit, x_tr_done), t_learn = timed(learned)
    t_learn_te = sum(i_te[k]["seconds"] for k in range(0, len(i_te), 64))
    # the library solves in chunks of up to 64 right-hand sides and reports
    # each chunk's time on its entries
    t_tr_solve = sum(i_tr[k]["seconds"] for k in range(0, len(i_tr), 64))
    print("sweep: span projection inside the sweep", file=sys.stderr, flush=True)
    (i_spi, spi_parts), t_spi = timed(lambda: span_in_sweep(x_tr_done))
    spi_parts["training_solve_s"] = round(t_tr_solve, 3)
    t_spi += t_tr_solve
    ok = all(i["converged"] for i in i_plain + i_batch + i_mixed + i_tr + i_te + i_mid + i_am + i_sp + i_spi)
    assert len(i_tr) + len(i_te) == n_ang
    ms = lambda t: round(1e3 * t / n_ang, 2)  # noqa: E731
    res_max = max(i["true_residual"] for i in i_plain + i_batch + i_mixed + i_tr + i_te + i_am + i_sp)
    out = {
        "angles": n_ang, "tol": 1e-4,
        "plain_timed_on": f"{len(plain_idx)} of {n_ang} angles (every {plain_stride}-th), scaled to the sweep",
        "ms_per_angle": {"plain_fp32": ms(t_plain), "batched_bf16split": ms(t_mixed),
                         "batched_bf16split_learned_in_sweep": ms(t_learn),
                         "batched_bf16split_span_projection_in_sweep": ms(t_spi)},
        "speedup_vs_plain": {"batched_bf16split": round(t_plain / t_mixed, 2),
                             "batched_bf16split_learned_in_sweep": round(t_plain / t_learn, 2),
                             "batched_bf16split_span_projection_in_sweep": round(t_plain / t_spi, 2)},
        "iterations_mean_max": {"plain_fp32": its(i_plain), "batched_bf16split": its(i_mixed),
                                "in_sweep_training_angles": its(i_tr), "in_sweep_predicted_angles": its(i_te),
                                "span_projection_in_sweep_predicted_angles": its(i_spi)},
        "true_residual_max": res_max,
        "guess_in_sweep": {"trained_on": len(tr), "fit_and_predict_s": round(t_fit, 3), "loss": loss,
                           "training_solve_s": round(sum(i_tr[k]["seconds"] for k in range(0, len(i_tr), 64)), 3),
                           "predicted_solve_s": round(t_learn_te, 3),
                           "initial_residual_median": float(np.median([i["initial_residual"] for i in i_te])),
                           "initial_residual_max": float(max(i["initial_residual"] for i in i_te)),
                           "used": int(sum(i["guess_used"] for i in i_te))},
        "span_projection_in_sweep": {
            "timed_as": "the learned run's training solves + fit without Adam steps + span guess + solve",
            "parts_s": spi_parts,
            "initial_residual_median": float(np.median([i["initial_residual"] for i in i_spi])),
            "initial_residual_max": float(max(i["initial_residual"] for i in i_spi))},
        "all_converged": bool(ok),
    }
    if batched_fp32:
        out["ms_per_angle"]["batched_fp32"] = ms(t_batch)
        out["speedup_vs_plain"]["batched_fp32"] = round(t_plain / t_batch, 2)
        out["iterations_mean_max"]["batched_fp32"] = its(i_batch)
    if pretrained:
        out["ms_per_angle"]["batched_bf16split_learned_pretrained"] = ms(t_am)
        out["ms_per_angle"]["batched_bf16split_span_projection_pretrained"] = ms(t_sp)
        out["speedup_vs_plain"]["batched_bf16split_learned_pretrained"] = round(t_plain / t_am, 2)
        out["speedup_vs_plain"]["batched_bf16split_span_projection_pretrained"] = round(t_plain / t_sp, 2)
        out["iterations_mean_max"]["pretrained"] = its(i_am)
        out["iterations_mean_max"]["span_projection_pretrained"] = its(i_sp)
        out["guess_pretrained"] = {
            "trained_on": len(mid), "coarse_solve_and_fit_s": round(t_pre, 3), "loss": loss_pre,
            "initial_residual_median": float(np.median([i["initial_residual"] for i in i_am])),
            "used": int(sum(i["guess_used"] for i in i_am))}
        out["span_projection_pretrained"] = {
            "initial_residual_median": float(np.median([i["initial_residual"] for i in i_sp])),
            "used": int(sum(i["guess_used"] for i in i_sp))}
    return out


def stage_profile(ctx, torch, x, y, reps, precond=True):
    ctx.sfmm_profile(1)
    for _ in range(reps):
        ctx.sfmm_matvec(x, y)
        if precond:
            ctx.sfmm_precond(x, y)
    torch.cuda.synchronize()
    st, _ = ctx.sfmm_profile(0)
    names = ["near", "aggregate", "interp_up", "translate", "anterp_down", "receive", "precond", "matvec_total"]
    return {k: round(float(v), 4) for k, v in zip(names, st)}


def mfma_utilisation(desc, pb, stages, R, split):
    """Useful flops of the R-RHS matrix-core products over their HIP-event
    stage times (the library reports stage times per right-hand side): near
    field 4 complex MACs (32 flops) per edge pair and right-hand side;
    aggregation and receive 4 complex MACs per region edge, direction and
    right-hand side each, i.e. (pattern bytes / 32) x 32 flops.  bf16-split
    counts its three bf16 products per FP32 product against the bf16 peak;
    FP32 against the FP32 matrix-core peak."""
    near_flops = 32.0 * desc["near_pairs"]         # per right-hand side
    agg_flops = float(pb["patterns"])              # (patterns / 32 B) x 32 flops, FP32 tables
    out = {}
    for name, flops, ms_ in (("near", near_flops, stages["near"]), ("aggregate", agg_flops / 2, stages["aggregate"]),
                             ("receive", agg_flops / 2, stages["receive"])):
        if ms_ <= 0:
            continue
        if split and name == "near":
            tf = 3 * flops / (ms_ * 1e-3) / 1e12
            peak = MFMA_PEAK_TFLOPS["bf16"]
        else:
            tf = flops / (ms_ * 1e-3) / 1e12
            peak = MFMA_PEAK_TFLOPS["fp32"]
        out[name] = {"tflops": round(tf, 2), "peak_tflops": peak, "frac": round(tf / peak, 4),
                     "ms_per_product": round(ms_ * R, 4), "rhs": R}
    return out


def coated_leg(sfmm, torch, stream, opts, n_ang, every, plain_stride):
    """The paper's multi-layer example at full size: 64-RHS bf16-split
    products and the 64-angle sweep, in one bf16-split context (its
    single-RHS products run the FP32 vector kernels, so its single-RHS
    solves are the plain FP32 path)."""
    from workloads import coated_sphere_body, random_complex_vector

    coated = coated_sphere_body(1.5, 6 - 0.5j, 5, 2.5, 2.56, 6)
    copts = dict(opts, poly_degree=48, n_levels=0, precision=sfmm.PREC_BF16_SPLIT)
    t0 = time.perf_counter()
    ctx = sfmm.Context([coated], **copts)
    setup_s = time.perf_counter() - t0
    ctx.sfmm_set_stream(stream.cuda_stream)
    n = ctx.sfmm_num_unknowns()
    print(f"coated sphere setup {setup_s:.1f} s, {n} unknowns", file=sys.stderr, flush=True)
    out = {"body": "two-layer coated sphere: core r=1.5 lambda0 eps_r 6-0.5j (s=5), shell r=2.5 lambda0 eps_r 2.56 "
                   "(s=6), 307,200 unknowns, 0.25 lambda0 boxes, 3 digits, bf16-split, polynomial "
                   "preconditioner degree 48", "setup_s": round(setup_s, 1)}
    xr = torch.from_numpy(random_complex_vector(n, 64, seed=99)).to("cuda")
    yr = torch.zeros_like(xr)
    ctx.sfmm_matvec(xr, yr)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(3):
        ctx.sfmm_matvec(xr, yr)
    e1.record()
    torch.cuda.synchronize()
    ms64 = e0.elapsed_time(e1) / 3
    out["product_64rhs_ms"] = round(ms64, 2)
    out["product_64rhs_unknowns_rhs_per_s"] = n * 64 / (ms64 * 1e-3)
    desc = ctx.sfmm_describe()
    pb = ctx.sfmm_product_bytes()
    st64 = stage_profile(ctx, torch, xr, yr, 2, precond=False)
    out["stages_ms_64rhs"] = st64
    out["mfma_64rhs"] = mfma_utilisation(desc, pb, st64, 64, split=True)
    del xr, yr
    print("coated 64-RHS product", out["product_64rhs_ms"], "ms", file=sys.stderr, flush=True)
    out["sweep"] = sweep(ctx, ctx, torch, n_ang, every, plain_stride=plain_stride, batched_fp32=False,
                         pretrained=False)
    ctx.close()
    return out


def cylinder_leg(sfmm, torch, stream, n_ang, every, plain_stride):
    """The three-layer stacked cylinder (junction edges, eps_r 2.2 / 4.4 /
    10.2, 82,080 unknowns) under JMCFIE with ILU(0): a monostatic theta sweep
    to 1e-4, plain single-RHS FP32 solves against batched FP32 and
    bf16-split solves and the learned guess trained on every `every`-th
    angle (zero-guess GMRES is the batched bf16-split solve)."""
    from workloads import stacked_cylinder_body

    body = stacked_cylinder_body(1.0, 3.0, (2.2, 4.4, 10.2), 0.05)
    opts = dict(formulation=sfmm.FORM_JMCFIE, preconditioner=sfmm.PRECOND_ILU0, finest_box=0.25, digits=3.0,
                gmres_restart=50, tol=1e-4, max_iters=1000)
    t0 = time.perf_counter()
    ctx = sfmm.Context([body], precision=sfmm.PREC_FP32, **opts)
    ctx_mixed = sfmm.Context([body], precision=sfmm.PREC_BF16_SPLIT, **opts)
    setup_s = time.perf_counter() - t0
    for c in (ctx, ctx_mixed):
        c.sfmm_set_stream(stream.cuda_stream)
    out = {"body": "three-layer stacked cylinder r=1 lambda0, h=3 lambda0, eps_r 2.2/4.4/10.2, mean edge "
                   "0.05 lambda0, 82,080 unknowns (252 junction edges), JMCFIE, ILU(0), 0.25 lambda0 boxes, "
                   "3 digits", "setup_s_both_contexts": round(setup_s, 1)}
    print(f"cylinder setup {setup_s:.1f} s", file=sys.stderr, flush=True)
    out["sweep"] = sweep(ctx, ctx_mixed, torch, n_ang, every, plain_stride=plain_stride, batched_fp32=True,
                         pretrained=False)
    ctx_mixed.close()
    ctx.close()
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU only: the path runs on a single MI355X, --gpus must be 1"}))
        sys.exit(2)
    if args.product_rhs != 1 and (not args.product_only or not 1 <= args.product_rhs <= 64):
        sys.exit("--product-rhs takes 1..64 and goes with --product-only")
    import torch

    from paper_1704_06862_amd import sfmm
    from workloads import random_complex_vector, sphere_body

    body = sphere_body(2.0, 2.56, 5)
    xh = random_complex_vector(2 * 30720, 1, seed=1234)
    cpu = None
    if not args.no_cpu_baseline and not args.product_only:
        # host-only work first, before this process touches the GPU (the
        # oracle's worker processes are forked from it)
        print("cpu baseline", file=sys.stderr, flush=True)
        cpu = cpu_baseline(body, xh[0], args.cpu_seconds)
    opts = dict(finest_box=0.25, n_levels=5, digits=3.0, extra_multipoles=0, precision=sfmm.PREC_FP32,
                gmres_restart=50, max_iters=1000, tol=1e-4, preconditioner=sfmm.PRECOND_POLY, poly_degree=16)
    t0 = time.perf_counter()
    ctx = sfmm.Context([body], **dict(opts, graphs=0 if args.no_graphs else 1))
    setup_s = time.perf_counter() - t0
    n = ctx.sfmm_num_unknowns()
    desc = ctx.sfmm_describe()
    print(f"setup {setup_s:.1f} s, {n} unknowns, {desc['finest_boxes']} finest boxes, "
          f"{desc['near_pairs']} near edge pairs", file=sys.stderr, flush=True)

    stream = torch.cuda.current_stream()
    ctx.sfmm_set_stream(stream.cuda_stream)
    assert xh.shape[1] == n
    if args.product_rhs != 1:
        xh = random_complex_vector(n, args.product_rhs, seed=99)
    x = torch.from_numpy(xh).to("cuda")
    y = torch.zeros_like(x)
    for _ in range(args.warmup):
        ctx.sfmm_matvec(x, y)
    torch.cuda.synchronize()
    # the library launches on `stream`; HIP events recorded on it bracket the
    # timed products
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        ctx.sfmm_matvec(x, y)
    e1.record(stream)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms = 1e3 * dt / args.steps
    ev_ms = e0.elapsed_time(e1) / args.steps
    value = n * args.steps / dt
    print(f"matvec {ms:.3f} ms (HIP events {ev_ms:.3f} ms)", file=sys.stderr, flush=True)
    if args.product_only:
        if args.copy_calibration > 0:
            a = torch.ones(args.copy_calibration * (1 << 18), dtype=torch.float32, device="cuda")
            c = torch.empty_like(a)
            for _ in range(3):
                c.copy_(a)
            torch.cuda.synchronize()
        print(json.dumps({"ms_per_step": ms, "hip_event_ms": ev_ms, "steps": args.steps, "warmup": args.warmup,
                          "rhs": args.product_rhs}))
        return

    # batched products (outside the timed region): unknowns x RHS per second
    batched = {}
    for R in [int(v) for v in args.batch.split(",") if v]:
        xr = torch.from_numpy(random_complex_vector(n, R, seed=99)).to("cuda")
        yr = torch.zeros_like(xr)
        ctx.sfmm_matvec(xr, yr)
        torch.cuda.synchronize()
        reps = max(2, 20 // R)
        t1 = time.perf_counter()
        for _ in range(reps):
            ctx.sfmm_matvec(xr, yr)
        torch.cuda.synchronize()
        batched[str(R)] = n * R * reps / (time.perf_counter() - t1)
        del xr, yr
    print("batched", batched, file=sys.stderr, flush=True)

    # per-stage HIP-event times (outside the timed region; stage-timed
    # products run kernel by kernel)
    stages = stage_profile(ctx, torch, x, y, 10)
    print("stages ms", stages, file=sys.stderr, flush=True)
    xr = torch.from_numpy(random_complex_vector(n, 64, seed=99)).to("cuda")
    yr = torch.zeros_like(xr)
    stages64 = stage_profile(ctx, torch, xr, yr, 3)
    print("stages ms at 64 RHS", stages64, file=sys.stderr, flush=True)
    pb = ctx.sfmm_product_bytes()
    mfma = {"fp32": mfma_utilisation(desc, pb, stages64, 64, split=False)}

    def gbs(nbytes, ms_):
        return nbytes / (ms_ * 1e-3) / 1e9 if ms_ > 0 else 0.0

    # a plain 1 GiB device-to-device copy (read + write) for the bandwidth the
    # chip reaches in practice, quoted beside the published peak
    src = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record()
    for _ in range(10):
        dst.copy_(src)
    c1.record()
    torch.cuda.synchronize()
    copy_gbs = 2 * (1 << 30) * 10 / (c0.elapsed_time(c1) * 1e-3) / 1e9
    del src, dst

    # roofline of the whole product: one replayed product (the HIP graph of
    # every stage's kernels) is the unit.  Algorithmic bytes (the library's
    # count of the stored-table form's least traffic, every array read or
    # written once per use) over its HIP-event time in the timed region.
    traffic, traffic_src = measured_traffic()
    achieved = gbs(pb["total"], ev_ms)
    roofline = {"bound": "hbm", "kernel": "whole MLFMM product (one HIP-graph replay: near field, aggregation, "
                                          "interpolation, translation, anterpolation, receive)",
                "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "traffic_source": traffic_src,
                "alg_bytes_per_launch": int(pb["total"]), "alg_bytes": pb, "avg_ms": round(ev_ms, 4),
                "avg_ms_measured": "HIP events on the library stream around the timed products",
                "measured_copy_GBs": round(copy_gbs, 1),
                "frac_of_measured_copy": round(achieved / copy_gbs, 4),
                "near_field_alone": {"alg_bytes": int(pb["near"] + pb["x_y"]), "ms": stages["near"],
                                     "achieved": round(gbs(pb["near"] + pb["x_y"], stages["near"]), 1)}}

    result = {"metric": METRIC, "value": value, "unit": "unknowns*RHS/s", "n_gpus": 1, "steps": args.steps,
              "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
              "vs_baseline": None, "dtype": "f32", "data": "synthetic",
              "config": {"workload": "dielectric sphere r=2 lambda0, eps_r=2.56, icosphere s=5, 61,440 unknowns, "
                                     "5-level MLFMM, 0.25 lambda0 boxes, 3 digits, FP32, 1 RHS"},
              "setup_s": round(setup_s, 2), "stages_ms": stages, "stages_ms_64rhs": stages64, "roofline": roofline,
              "batched_unknowns_rhs_per_s": batched}

    if not args.no_solve:
        b = torch.zeros_like(x)
        ctx.sfmm_planewave_rhs(np.array([[0.0, 0.0]]), b)
        xs = torch.zeros_like(x)
        torch.cuda.synchronize()
        info = ctx.sfmm_solve(b, xs)[0]
        result["gmres"] = {"time_to_1e-4_ms": round(1e3 * info["seconds"], 2), "iterations": info["iterations"],
                           "restart": 50, "true_residual": info["true_residual"], "converged": info["converged"],
                           "preconditioner": "near-field GMRES polynomial, degree 16"}
        print("gmres", result["gmres"], file=sys.stderr, flush=True)

    ctx_mixed = sfmm.Context([body], **dict(opts, precision=sfmm.PREC_BF16_SPLIT))
    ctx_mixed.sfmm_set_stream(stream.cuda_stream)
    st_bf = stage_profile(ctx_mixed, torch, xr, yr, 3, precond=False)
    mfma["bf16split"] = mfma_utilisation(desc, pb, st_bf, 64, split=True)
    result["mfma_64rhs"] = mfma
    del xr, yr
    if args.sweep > 0:
        result["sweep"] = sweep(ctx, ctx_mixed, torch, args.sweep, args.train_every)
        print("sweep", result["sweep"], file=sys.stderr, flush=True)
    ctx_mixed.close()
    ctx.close()
    if args.sweep > 0 and not args.no_coated:
        result["coated"] = coated_leg(sfmm, torch, stream, opts, args.sweep, args.train_every,
                                      args.coated_plain_stride)
        print("coated", result["coated"], file=sys.stderr, flush=True)

    if args.cylinder_sweep > 0:
        result["cylinder"] = cylinder_leg(sfmm, torch, stream, args.cylinder_sweep, args.cylinder_train_every,
                                          args.cylinder_plain_stride)
        print("cylinder", result["cylinder"], file=sys.stderr, flush=True)

    if args.copy_calibration > 0:
        a = torch.ones(args.copy_calibration * (1 << 18), dtype=torch.float32, device="cuda")
        c = torch.empty_like(a)
        for _ in range(3):
            c.copy_(a)
        torch.cuda.synchronize()
        del a, c

    if cpu is not None:
        result["cpu_baseline"] = cpu
    print(json.dumps(result))


if __name__ == "__main__":
    main()
