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
count), the roofline of the dominant kernel, and the CPU oracle on a bounded
row sample.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "MLFMM matvec unknowns×RHS/s + GMRES time-to-1e-4 per angle vs plain GPU path"
HBM_PEAK_GBS = 8000.0
# HBM bytes of one k_near launch at this size from rocprofv3 --pmc: FETCH_SIZE
# (KiB) x 2.0 + WRITE_SIZE (KiB) x 1.0, the factors being what the counters
# read for a plain 256 MiB device copy (profiles/near_product_sphere61440_pmc_traffic.md)
NEAR_TRAFFIC_BYTES = int((157493 * 2.0 + 568) * 1024)


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
    p.add_argument("--sweep-body", choices=["sphere", "coated"], default="sphere",
                   help="body of the sweep: the benchmark sphere, or the two-layer coated sphere (lossy core "
                        "r = 1.5, eps 6-0.5j, s = 5; shell r = 2.5, eps 2.56, s = 6; 307,200 unknowns; "
                        "degree-48 polynomial preconditioner); the coated sweep takes several minutes")
    p.add_argument("--copy-calibration", type=int, default=0,
                   help="MiB of a plain device copy run after the measurements, to scale HBM byte counters")
    return p.parse_args()


def cpu_baseline(body, x, seconds):
    """Oracle rows of Z x (E and H rows of sampled edges) for ~seconds of CPU."""
    from threadpoolctl import threadpool_limits

    from oracle import mom, rwg

    mesh = rwg.from_body(body)
    rng = np.random.default_rng(0)
    order = rng.permutation(mesh.n_edges)
    done = 0
    t0 = time.perf_counter()
    with threadpool_limits(limits=1):
        while time.perf_counter() - t0 < seconds and done < len(order):
            e = order[done: done + 2]
            ZE, ZH = mom.pmchwt_rows(mesh, body.eps_r, body.mu_r, body.frequency, e)
            _ = ZE @ x, ZH @ x
            done += len(e)
    dt = time.perf_counter() - t0
    rows = 2 * done
    # one full product needs 2E rows: unknowns x RHS per second = rows / s
    return {"value": rows / dt, "unit": "unknowns*RHS/s", "cores": 1, "kind": "oracle",
            "sample": f"{rows} of {2 * mesh.n_edges} rows of Z x (dense PMCHWT rows with singular "
                      f"extraction, FP64 numpy, 1 thread) in {dt:.1f} s"}


def sweep(ctx, ctx_mixed, torch, n_ang, every):
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
    i_plain, t_plain = timed(lambda: [plain_one(i) for i in range(n_ang)])
    print("sweep: batched solves", file=sys.stderr, flush=True)
    x.zero_()
    i_batch, t_batch = timed(lambda: ctx.sfmm_solve(b, x))
    x.zero_()
    i_mixed, t_mixed = timed(lambda: ctx_mixed.sfmm_solve(b, x))

    tr = np.arange(0, n_ang, every)
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
        return i_tr, i_te, loss, t_fit

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

    (i_tr, i_te, loss, t_fit), t_learn = timed(learned)
    ok = all(i["converged"] for i in i_plain + i_batch + i_mixed + i_tr + i_te + i_mid + i_am + i_sp)
    assert len(i_tr) + len(i_te) == n_ang
    ms = lambda t: round(1e3 * t / n_ang, 2)  # noqa: E731
    return {
        "angles": n_ang, "tol": 1e-4,
        "ms_per_angle": {"plain_fp32": ms(t_plain), "batched_fp32": ms(t_batch), "batched_bf16split": ms(t_mixed),
                         "batched_bf16split_learned_in_sweep": ms(t_learn),
                         "batched_bf16split_learned_pretrained": ms(t_am),
                         "batched_bf16split_span_projection_pretrained": ms(t_sp)},
        "speedup_vs_plain": {"batched_fp32": round(t_plain / t_batch, 2),
                             "batched_bf16split": round(t_plain / t_mixed, 2),
                             "batched_bf16split_learned_in_sweep": round(t_plain / t_learn, 2),
                             "batched_bf16split_learned_pretrained": round(t_plain / t_am, 2),
                             "batched_bf16split_span_projection_pretrained": round(t_plain / t_sp, 2)},
        "iterations_mean_max": {"plain_fp32": its(i_plain), "batched_fp32": its(i_batch),
                            "batched_bf16split": its(i_mixed), "in_sweep_training_angles": its(i_tr),
                            "in_sweep_predicted_angles": its(i_te),
                            "pretrained": its(i_am),
                            "span_projection_pretrained": its(i_sp)},
        "true_residual_max": max(i["true_residual"] for i in i_plain + i_batch + i_mixed + i_tr + i_te + i_am + i_sp),
        "guess_in_sweep": {"trained_on": len(tr), "fit_and_predict_s": round(t_fit, 3), "loss": loss,
                           "initial_residual_median": float(np.median([i["initial_residual"] for i in i_te])),
                           "used": int(sum(i["guess_used"] for i in i_te))},
        "guess_pretrained": {"trained_on": len(mid), "coarse_solve_and_fit_s": round(t_pre, 3), "loss": loss_pre,
                             "initial_residual_median": float(np.median([i["initial_residual"] for i in i_am])),
                             "used": int(sum(i["guess_used"] for i in i_am))},
        "span_projection_pretrained": {
            "initial_residual_median": float(np.median([i["initial_residual"] for i in i_sp])),
            "used": int(sum(i["guess_used"] for i in i_sp))},
        "all_converged": bool(ok),
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    import torch

    from paper_1704_06862_amd import sfmm
    from workloads import random_complex_vector, sphere_body

    body = sphere_body(2.0, 2.56, 5)
    opts = dict(finest_box=0.25, n_levels=5, digits=3.0, extra_multipoles=0, precision=sfmm.PREC_FP32,
                gmres_restart=50, max_iters=1000, tol=1e-4, preconditioner=sfmm.PRECOND_POLY, poly_degree=16)
    t0 = time.perf_counter()
    ctx = sfmm.Context([body], **opts)
    setup_s = time.perf_counter() - t0
    n = ctx.sfmm_num_unknowns()
    desc = ctx.sfmm_describe()
    print(f"setup {setup_s:.1f} s, {n} unknowns, {desc['finest_boxes']} finest boxes, "
          f"{desc['near_pairs']} near edge pairs", file=sys.stderr, flush=True)

    stream = torch.cuda.current_stream()
    ctx.sfmm_set_stream(stream.cuda_stream)
    xh = random_complex_vector(n, 1, seed=1234)
    x = torch.from_numpy(xh).to("cuda")
    y = torch.zeros_like(x)
    for _ in range(args.warmup):
        ctx.sfmm_matvec(x, y)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.sfmm_matvec(x, y)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms = 1e3 * dt / args.steps
    value = n * args.steps / dt
    print(f"matvec {ms:.3f} ms", file=sys.stderr, flush=True)

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

    # per-stage HIP-event times (outside the timed region)
    ctx.sfmm_profile(1)
    for _ in range(10):
        ctx.sfmm_matvec(x, y)
        ctx.sfmm_precond(x, y)
    torch.cuda.synchronize()
    st, cnt = ctx.sfmm_profile(0)
    names = ["near", "aggregate", "interp_up", "translate", "anterp_down", "receive", "precond", "matvec_total"]
    stages = {k: round(float(v), 4) for k, v in zip(names, st)}
    print("stages ms", stages, file=sys.stderr, flush=True)
    # the same at 64 right-hand sides (one batched product / application)
    xr = torch.from_numpy(random_complex_vector(n, 64, seed=99)).to("cuda")
    yr = torch.zeros_like(xr)
    ctx.sfmm_profile(1)
    for _ in range(3):
        ctx.sfmm_matvec(xr, yr)
        ctx.sfmm_precond(xr, yr)
    torch.cuda.synchronize()
    st64, _ = ctx.sfmm_profile(0)
    stages64 = {k: round(float(v), 4) for k, v in zip(names, st64)}
    del xr, yr
    print("stages ms at 64 RHS", stages64, file=sys.stderr, flush=True)

    # dominant kernel roofline: the near-field product (one kernel launch).
    # Algorithmic bytes per launch (from the library's own tables): 3 complex
    # FP32 values per edge pair, one int32 column index per (box, column), x
    # read once, y written once.
    pb = ctx.sfmm_product_bytes()
    alg_bytes = pb["near"] + pb["x_y"]

    def gbs(nbytes, ms_):
        return nbytes / (ms_ * 1e-3) / 1e9 if ms_ > 0 else 0.0

    # a plain 1 GiB device-to-device copy (read + write) for the bandwidth the
    # chip reaches in practice, quoted beside the published peak
    src = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 2 * (1 << 30) * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst

    near_ms = st[0]
    achieved = gbs(alg_bytes, near_ms)
    roofline = {"bound": "hbm", "kernel": "k_near (near-field box-ELL product)", "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": NEAR_TRAFFIC_BYTES, "alg_bytes_per_launch": int(alg_bytes), "avg_ms": round(near_ms, 4),
                "avg_ms_measured": "HIP events on the library stream around k_near in 10 products launched kernel by "
                                   "kernel; the graph the timed steps replay runs the same rows as the trailing "
                                   "workgroups of the level-2 translation launch (k_near_up_phi1_translate1<float, "
                                   "true>), overlapped with that level's translations",
                "measured_copy_GBs": round(copy_gbs, 1),
                "whole_product": {"alg_bytes": pb, "ms": round(ms, 4), "achieved": round(gbs(pb["total"], ms), 1),
                                  "frac": round(gbs(pb["total"], ms) / HBM_PEAK_GBS, 4)}}

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

    if args.sweep > 0 and args.sweep_body == "sphere":
        ctx_mixed = sfmm.Context([body], **dict(opts, precision=sfmm.PREC_BF16_SPLIT))
        ctx_mixed.sfmm_set_stream(stream.cuda_stream)
        result["sweep"] = sweep(ctx, ctx_mixed, torch, args.sweep, args.train_every)
        ctx_mixed.close()
        print("sweep", result["sweep"], file=sys.stderr, flush=True)
    elif args.sweep > 0:
        from workloads import coated_sphere_body

        ctx.close()
        coated = coated_sphere_body(1.5, 6 - 0.5j, 5, 2.5, 2.56, 6)
        copts = dict(opts, poly_degree=48, n_levels=0)   # the 2.5-wavelength shell needs a deeper tree
        t0 = time.perf_counter()
        ctx_c = sfmm.Context([coated], **copts)
        ctx_cm = sfmm.Context([coated], **dict(copts, precision=sfmm.PREC_BF16_SPLIT))
        for c in (ctx_c, ctx_cm):
            c.sfmm_set_stream(stream.cuda_stream)
        print(f"coated sphere setup {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
        result["sweep"] = sweep(ctx_c, ctx_cm, torch, args.sweep, args.train_every)
        result["sweep"]["body"] = ("two-layer coated sphere: core r=1.5 lambda0 eps_r 6-0.5j (s=5), shell r=2.5 "
                                   "lambda0 eps_r 2.56 (s=6), 307,200 unknowns, 0.25 lambda0 boxes, polynomial "
                                   "preconditioner degree 48")
        ctx_c.close()
        ctx_cm.close()
        print("sweep", result["sweep"], file=sys.stderr, flush=True)

    if args.copy_calibration > 0:
        a = torch.ones(args.copy_calibration * (1 << 18), dtype=torch.float32, device="cuda")
        c = torch.empty_like(a)
        for _ in range(3):
            c.copy_(a)
        torch.cuda.synchronize()
        del a, c

    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(body, xh[0], args.cpu_seconds)
    ctx.close()
    print(json.dumps(result))


if __name__ == "__main__":
    main()
