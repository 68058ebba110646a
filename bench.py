"""Benchmark of the rational-program hot path on one MI355X.

One step = one pass of the whole path over one batch of synthetic input:
  1. fit the batched workload: 4096 fits over (n, bx, by), degree 3/3
     (20 + 19 unknowns), 2048 samples each -- Gram with on-chip design
     assembly, per-fit FP64 sweep inverse, FP64 refinement (rp_fit_rational);
  2. one step of true-loss refinement of every fit: the FP32 adjoint forward
     and backward (rp_loss_grad) and one FP64 Levenberg-Marquardt step
     (rp_refine_rational, max_iter = 1);
  3. evaluate the 16-metric MWP-CWP program at 1024 data sizes for all 230
     block formats and select the minimiser per data size with the evaluator
     generated for this program and compiled at set-up (rp_program_specialize,
     rp_eval_spec_select); the table-driven evaluator (rp_eval_program_argmin)
     is timed beside it.
Inputs are resident in HBM before timing starts.  ``value`` is fits/s of the
whole step (4096 fits / step time) in the fastest form; every form (plain FP64,
mixed FP32, mixed BF16) of the same step is timed and reported beside it.  The
timed step is one replay of a HIP graph holding every kernel of the four
stages, the program evaluation (which does not depend on the fits) and then
the adjoint (which needs only the fitted coefficients) on a branch of their
own beside the fit and LM chain; its outputs are checked bit for bit against
an eager step, and the
per-stage breakdown comes from eager steps with HIP events between the stages.

Prints one JSON line.  One GPU only: the fits are independent, and how the
batch would be split over several GPUs is a matter of partitioning the fit list.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# MI355X published peaks
PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6

# Adam learning rate of the differentiation workload's FP32 stage: from the
# linearised fit the true loss is already near its minimum in most directions,
# and larger rates overshoot along the stiff ones (see the learning-rate sweep
# that the diff report prints)
ADAM_LR = 1e-5


def moment_kernel_source_sha():
    """SHA-256 of the moment-Gram kernels' source: the section of
    rp_fit_kernels.h between its two section markers plus the moment-pair
    layout of rp_internal.h.  The committed traffic figures are valid for this
    hash."""
    import hashlib
    root = os.path.dirname(os.path.abspath(__file__))
    csrc = os.path.join(root, "paper_1906_00142_amd", "csrc")
    text = open(os.path.join(csrc, "rp_fit_kernels.h")).read()
    a = text.index("// FP64 Gram by weighted moments (VALU)")
    b = text.index("// split form, solve: block sweep", a)
    h = hashlib.sha256(text[a:b].encode())
    internal = open(os.path.join(csrc, "rp_internal.h")).read()
    a = internal.index("// Exponent table of any size")
    b = internal.index("// Shape of a linearised model", a)
    h.update(internal[a:b].encode())
    return h.hexdigest()


def committed_traffic(kernel):
    """HBM bytes per launch of `kernel` (a key of the committed counter
    summary), or None if the kernels' source changed since it was measured."""
    root = os.path.dirname(os.path.abspath(__file__))
    summ = os.path.join(root, "profiles", "k_gram_mom_batched4096.md")
    try:
        kv = dict(line.split(": ", 1) for line in open(summ).read().splitlines()
                  if line.startswith(("traffic_bytes_per_launch", "source_sha256:")))
        if kv.get("source_sha256", "").strip() != moment_kernel_source_sha():
            return None
        return float(kv[f"traffic_bytes_per_launch[{kernel}]"])
    except (OSError, KeyError, ValueError):
        return None


def moment_pairs(v, d, jacobian):
    """Moment-weight pairs per sample of the FP64 Gram by moments: weights 1,
    y, y^2 at every exponent of degree <= 2d (linear problem).  The Jacobian
    form's weights 1/Q^2, f/Q^2, f^2/Q^2, r/Q, f r/Q, r^2 are needed only
    where an entry of the Gram uses them: the constant takes 1/Q^2, r/Q, r^2;
    the v exponents of degree 1 take 1/Q^2, f/Q^2, r/Q, f r/Q; degree 2..d all
    but r^2; degree d+1..2d the first three."""
    from math import comb
    nm1, nm2 = comb(v + d, d), comb(v + 2 * d, 2 * d)
    if not jacobian:
        return 3 * nm2
    return 3 + 4 * v + 5 * (nm1 - 1 - v) + 3 * (nm2 - nm1)


def _timed(fn, reps, stream):
    """Average milliseconds of fn() over reps launches, HIP events on stream."""
    import torch
    for _ in range(2):
        fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def report(args):
    """The workloads other than the batched step, each measured on its own
    (inputs resident, HIP events) and checked against the oracle, one JSON
    line each:
      tiny     1 fit of 256 samples (degree 2/2 over n, b), then evaluation and
               argmin over 32 block sizes at 64 data sizes: us per fit and per
               argmin (launch latency, not a roofline case);
      program  the MWP-CWP program over 1024 data sizes x 230 block formats:
               evaluations/s of the table-driven FP64 and FP32 evaluators and
               of the specialised one, FP32-vs-FP64 selection agreement;
      diff     4096 fits x 2048 samples, degree 3/3: 200 Adam iterations on
               the FP32 adjoint then one FP64 Levenberg-Marquardt step:
               iterations/s and the adjoint kernel's HBM rate;
      uneven   16384 fits of mixed sizes, shapes and degrees as one graph
               launch per form, then every fitted model evaluated over 4096
               candidates at 4 data sizes: fits/s per form, evaluations/s."""
    import torch
    import oracle
    from paper_1906_00142_amd import rp
    from paper_1906_00142_amd import workloads as W

    dev = torch.device("cuda", 0)
    ctx = rp.Context(0)
    stream = torch.cuda.current_stream()
    which = ["tiny", "program", "diff", "uneven"] if args.report == "all" else [args.report]
    reps = max(args.steps, 10)

    def emit(d):
        print(json.dumps(d), flush=True)

    if "tiny" in which:
        b = W.tiny_fit()
        db = rp.DeviceBatch(ctx, b)
        coef, status, resid, iters = db.fit()
        deg = np.array([2], np.int32)
        prog = rp.Program(ctx, rp.RP_TEMPLATE_SINGLE, 2, deg, deg, db.plan.coef_off, coef,
                          [2.0 ** 14, 1024.0])
        n_grid = W.tiny_grid(64)
        n_t = torch.from_numpy(n_grid).to(dev)
        cand = (32 * np.arange(1, 33)).astype(np.int32).reshape(-1, 1)
        c_t = torch.from_numpy(cand).to(dev)
        am = torch.empty((1, 64), dtype=torch.int32, device=dev)
        best = torch.empty((1, 64), dtype=torch.float64, device=dev)
        second = torch.empty_like(best)
        fit_ms = _timed(lambda: db.fit(out=(coef, status, resid, iters)), reps * 10, stream)
        ev_ms = _timed(lambda: rp.rp_eval_program_argmin(prog, n_t, c_t, am, best, second), reps * 10, stream)
        out = db.alloc_fit_outputs()
        g = rp.FitGraph(db, *out)
        graph_ms = _timed(lambda: g.launch(), reps * 10, stream)
        u, y = b.fit_samples(0)
        oc, ost, ork, ors = oracle.fit(u, y, 2, 2)
        c = coef.cpu().numpy()
        oprog = oracle.Program(oracle.TEMPLATE_SINGLE, 2, deg, deg, oc, [0, len(oc)], scale=[2.0 ** 14, 1024.0])
        oam, obest, _ = oracle.argmin(oprog, n_grid, cand)
        emit({"workload": "tiny: 1 fit x 256 samples, degree 2/2; argmin over 32 block sizes x 64 data sizes",
              "us_per_fit": fit_ms * 1e3, "us_per_fit_graph": graph_ms * 1e3, "us_per_argmin": ev_ms * 1e3,
              "coef_rel_err": float(np.max(np.abs(c - oc)) / np.max(np.abs(oc))),
              "same_argmin": int(np.sum(am.cpu().numpy() == oam)), "of": 64})
        g.close()

    if "program" in which:
        pw = W.program_workload()
        prog, n_t, cand_t = rp.program_from_workload(ctx, pw, dev)
        spec = rp.Spec(prog)
        P, nn, nc = 1, len(pw.n_grid), int(cand_t.shape[0])
        mk = lambda dt: torch.empty((P, nn), dtype=dt, device=dev)
        o64, o32, osp = [(mk(torch.int32), mk(torch.float64), mk(torch.float64)) for _ in range(3)]
        t64 = _timed(lambda: rp.rp_eval_program_argmin(prog, n_t, cand_t, *o64, precision=rp.RP_FP64), reps, stream)
        t32 = _timed(lambda: rp.rp_eval_program_argmin(prog, n_t, cand_t, *o32, precision=rp.RP_MIXED_FP32), reps, stream)
        tsp = _timed(lambda: rp.rp_eval_spec_select(spec, n_t, cand_t, *osp), reps, stream)
        evals = nn * nc
        flops = 1400.0 * evals
        same32 = int((o32[0] == o64[0]).sum().item())
        emit({"workload": "program: MWP-CWP, 16 metrics, 1024 data sizes x 230 block formats",
              "evals_per_launch": evals,
              "fp64_table": {"us": t64 * 1e3, "evals_per_s": evals / (t64 * 1e-3),
                             "frac_fp64_valu": flops / (t64 * 1e-3) / 1e12 / PEAK_FP64_TFLOPS},
              "fp32_scan_fp64_rescore": {"us": t32 * 1e3, "evals_per_s": evals / (t32 * 1e-3),
                                         "same_selection_as_fp64": same32, "of": nn,
                                         "best_max_rel_diff": float(((o32[1] - o64[1]).abs() / o64[1].abs()).max())},
              "fp64_specialised": {"us": tsp * 1e3, "evals_per_s": evals / (tsp * 1e-3),
                                   "same_selection_as_table": bool(torch.equal(osp[0], o64[0]))},
              "flops_per_eval_stated": 1400})

    if "diff" in which:
        b = W.refine_batch()
        db = rp.DeviceBatch(ctx, b)
        coef, status, resid, iters = db.fit()
        Fn = rp.rational_loss_function()
        ok = torch.from_numpy(np.where(status.cpu().numpy() == 0)[0]).to(dev)

        def adam_loss(lr, n=200):
            """Summed true loss (FP32 adjoint, fits fitted with status 0)
            after n Adam iterations from the linearised fit."""
            cc = coef.to(torch.float32).clone().requires_grad_(True)
            o = torch.optim.Adam([cc], lr=lr)
            for _ in range(n):
                o.zero_grad()
                Fn.apply(cc, db).sum().backward()
                o.step()
            return float(Fn.apply(cc, db).detach()[ok].double().sum())

        # the learning rate: the loss each rate reaches in 200 iterations
        lr_sweep = {f"{lr:g}": adam_loss(lr) for lr in (1e-3, 1e-4, 1e-5, 1e-6)}
        loss_lin = adam_loss(0.0, n=0)
        c = coef.to(torch.float32).clone().requires_grad_(True)
        opt = torch.optim.Adam([c], lr=ADAM_LR)

        def adam_iter():
            opt.zero_grad()
            Fn.apply(c, db).sum().backward()
            opt.step()
        for _ in range(3):
            adam_iter()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(200):
            adam_iter()
        e1.record(stream)
        torch.cuda.synchronize()
        adam_ms = e0.elapsed_time(e1)
        start = c.detach().to(torch.float64).contiguous()
        st = torch.zeros(b.num_fits, dtype=torch.int32, device=dev)
        loss = torch.zeros(b.num_fits, dtype=torch.float64, device=dev)
        s0 = start.clone()
        lm_ms = _timed(lambda: (start.copy_(s0), rp.rp_refine_rational(db.plan, db.x, db.ld_x, db.y, start, st,
                                                                         loss, max_iter=1)), reps, stream)
        loss32 = torch.empty(b.num_fits, dtype=torch.float32, device=dev)
        ones = torch.ones(b.num_fits, dtype=torch.float32, device=dev)
        dc = torch.empty_like(c)
        cc = c.detach().contiguous()
        bwd_ms = _timed(lambda: rp.rp_loss_grad(db.plan, db.x, db.ld_x, db.y, cc, loss32, ones, dc,
                                                mode=rp.RP_LOSS_BWD), reps, stream)
        fwd_ms = _timed(lambda: rp.rp_loss_grad(db.plan, db.x, db.ld_x, db.y, cc, loss32, mode=rp.RP_LOSS_FWD),
                        reps, stream)
        nbytes = float(b.total_samples) * 4 * 8
        loss_adam = float(Fn.apply(c.detach().clone(), db).detach()[ok].double().sum())
        start.copy_(s0)
        rp.rp_refine_rational(db.plan, db.x, db.ld_x, db.y, start, st, loss, max_iter=1)
        loss_lm1 = float(loss[ok].sum())
        start.copy_(s0)
        rp.rp_refine_rational(db.plan, db.x, db.ld_x, db.y, start, st, loss, max_iter=30)
        loss_lm30 = float(loss[ok].sum())
        emit({"workload": "diff: 4096 fits x 2048 samples, degree 3/3, 200 Adam iterations (FP32 adjoint) "
                          "+ one FP64 LM step",
              "adam_lr": ADAM_LR,
              "loss_sum_status0_fits": {"linearised_fit": loss_lin, "after_adam": loss_adam,
                                        "after_adam_and_one_lm_step": loss_lm1,
                                        "after_adam_and_30_lm_steps": loss_lm30,
                                        "after_200_adam_by_lr": lr_sweep},
              "adam_ms_200": adam_ms, "adam_iters_per_s": 200 / (adam_ms * 1e-3),
              "fit_iters_per_s": 200 * b.num_fits / (adam_ms * 1e-3),
              "lm_step_ms": lm_ms, "total_ms": adam_ms + lm_ms,
              "fits_per_s_total": b.num_fits / ((adam_ms + lm_ms) * 1e-3),
              "adjoint_fwd_us": fwd_ms * 1e3, "adjoint_bwd_us": bwd_ms * 1e3,
              "adjoint_bwd_hbm_gbs": nbytes / (bwd_ms * 1e-3) / 1e9,
              "adjoint_bwd_frac_hbm": nbytes / (bwd_ms * 1e-3) / 1e9 / PEAK_HBM_GBS})

    if "uneven" in which:
        b = W.uneven_batch()
        db = rp.DeviceBatch(ctx, b)
        forms = {}
        outs = {}
        t_tune = None
        for name in ("fp64", "fp32", "bf16", "auto"):
            if name == "auto":
                # per bucket, the form the tuner measures fastest
                t0 = time.perf_counter()
                rp.rp_plan_tune(db.plan, db.x, db.ld_x, db.y)
                t_tune = time.perf_counter() - t0
            out = db.alloc_fit_outputs()
            g = rp.FitGraph(db, *out, precision=rp.PRECISIONS[name])
            ms = _timed(lambda: g.launch(), max(args.steps, 5), stream)
            forms[name] = {"ms": ms, "fits_per_s": b.num_fits / (ms * 1e-3),
                           "status_counts": np.bincount(out[1].cpu().numpy(), minlength=6).tolist()}
            outs[name] = out
            g.close()
        tuning = rp.rp_plan_tuning(db.plan)
        # per bucket: fits, samples and the refinement steps each form took
        # (median over the bucket's fits; CG iterations for the mixed forms)
        buckets = []
        m_f = np.diff(b.sample_off)
        for r in tuning:
            idx = np.where((b.nvars == r[0]) & (b.deg_num == r[1]) & (b.deg_den == r[2]))[0]
            buckets.append({"nvars": int(r[0]), "deg_num": int(r[1]), "deg_den": int(r[2]),
                            "fits": int(len(idx)), "samples": int(m_f[idx].sum()),
                            "iters_median": {name: float(np.median(outs[name][3].cpu().numpy()[idx]))
                                             for name in ("fp64", "fp32", "bf16")}})
        # each bucket alone in each form (the tuner's own HIP-event timing),
        # against the whole graph: how much the buckets overlap
        bucket_sum = {k: int(tuning[:, 5 + i].sum()) for i, k in
                      enumerate(("fp64_moments", "fp64_mfma", "fp32", "bf16"))}
        bucket_sum["auto"] = int(tuning[:, 5:].min(axis=1).sum())
        bucket_max = {"auto": int(tuning[:, 5:].min(axis=1).max())}
        # every fitted model scored over 4096 candidates at 4 data sizes, one
        # program batch per variable count
        coef = outs["fp64"][0]
        n_grid = torch.tensor([1024.0, 2048.0, 3072.0, 4096.0], dtype=torch.float64, device=dev)
        ev = 0.0
        nev = 0
        coff = db.plan.coef_off
        for v in (2, 3, 4):
            idx = np.where(b.nvars == v)[0]
            if len(idx) == 0:
                continue
            g = {2: 4096, 3: 64, 4: 16}[v]
            mesh = np.meshgrid(*([np.arange(1, g + 1)] * (v - 1)), indexing="ij")
            cand = torch.from_numpy(np.stack([a.ravel() for a in mesh], axis=-1).astype(np.int32)).to(dev)
            sub = torch.cat([coef[int(coff[f]):int(coff[f + 1])] for f in idx])
            off = np.zeros(len(idx) + 1, np.int64)
            np.cumsum([int(coff[f + 1] - coff[f]) for f in idx], out=off[1:])
            deg = b.deg_num[idx].astype(np.int32)
            prog = rp.Program(ctx, rp.RP_TEMPLATE_SINGLE, v, deg, deg, off, sub,
                              [4096.0] + [float(g)] * (v - 1), num_programs=len(idx))
            am = torch.empty((len(idx), 4), dtype=torch.int32, device=dev)
            bb = torch.empty((len(idx), 4), dtype=torch.float64, device=dev)
            ss = torch.empty_like(bb)
            ev += _timed(lambda: rp.rp_eval_program_argmin(prog, n_grid, cand, am, bb, ss), 3, stream)
            nev += len(idx) * 4 * int(cand.shape[0])
        emit({"workload": "uneven: 16384 fits, m log-uniform [64, 8192], v in {2,3,4}, d in {1..4}, "
                          "one graph launch per form; evaluation over 4096 candidates x 4 data sizes",
              "total_samples": int(b.total_samples), "forms": forms,
              "buckets": buckets,
              "tuning": {"columns": rp.TUNE_COLUMNS, "rows": tuning.tolist(), "tune_s": t_tune,
                         "sum_of_buckets_alone_us": bucket_sum,
                         "longest_bucket_alone_us": bucket_max},
              "mixed_vs_fp64": forms["fp64"]["ms"] / min(forms["fp32"]["ms"], forms["bf16"]["ms"]),
              "auto_vs_fp64": forms["fp64"]["ms"] / forms["auto"]["ms"],
              "eval_ms": ev, "evals": nev, "evals_per_s": nev / (ev * 1e-3)})


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--fits", type=int, default=4096)
    ap.add_argument("--samples", type=int, default=2048)
    ap.add_argument("--forms", default="fp64,fp32,bf16")
    ap.add_argument("--cpu-sample", type=int, default=4096, help="fits timed on the CPU oracle")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-graph", action="store_true",
                    help="time the eager step (stage by stage on one stream) only")
    ap.add_argument("--max-refine", type=int, default=-1)
    ap.add_argument("--probe", choices=["gram", "solve", "mfma"], default=None,
                    help="counter run: only the dominant kernel and a reference copy")
    ap.add_argument("--report", choices=["tiny", "program", "diff", "uneven", "all"], default=None,
                    help="measure the other workloads instead (one JSON line each)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py measures one GPU only (no multi-GPU path); run with --gpus 1"}))
        sys.exit(2)
    if args.report:
        report(args)
        return

    import torch
    from paper_1906_00142_amd import rp
    from paper_1906_00142_amd import workloads as W

    dev = torch.device("cuda", 0)
    ctx = rp.Context(0)
    t0 = time.time()
    batch = W.batched_fit(num_fits=args.fits, num_samples=args.samples)
    pw = W.program_workload()
    log(f"workloads generated in {time.time() - t0:.1f}s")

    db = rp.DeviceBatch(ctx, batch)
    F = batch.num_fits
    NC = rp.rp_num_coefs(3, 3, 3)
    out = db.alloc_fit_outputs()
    loss32 = torch.empty(F, dtype=torch.float32, device=dev)
    dcoef32 = torch.empty(db.plan.num_coefs, dtype=torch.float32, device=dev)
    coef32 = torch.empty(db.plan.num_coefs, dtype=torch.float32, device=dev)
    ones = torch.ones(F, dtype=torch.float32, device=dev)
    gn_coef = torch.empty(db.plan.num_coefs, dtype=torch.float64, device=dev)
    gn_status = torch.empty(F, dtype=torch.int32, device=dev)
    gn_loss = torch.empty(F, dtype=torch.float64, device=dev)

    # program workload on the device; the evaluator specialised to it is
    # generated and compiled here, before any timing (the paper's code
    # generation precedes run time)
    prog, n_t, cand_t = rp.program_from_workload(ctx, pw, dev)
    t_spec = time.perf_counter()
    spec = rp.Spec(prog)
    compile_ms = (time.perf_counter() - t_spec) * 1e3
    am = torch.empty((1, len(pw.n_grid)), dtype=torch.int32, device=dev)
    best = torch.empty((1, len(pw.n_grid)), dtype=torch.float64, device=dev)
    second = torch.empty((1, len(pw.n_grid)), dtype=torch.float64, device=dev)

    forms = [f for f in args.forms.split(",") if f]
    stream = torch.cuda.current_stream()

    if args.probe == "gram":
        # For hardware-counter runs: three launches of each batched FP64 Gram
        # by moments (linear problem, then the Jacobian at the fitted
        # coefficients), then three device copies of a known 256 MiB buffer
        # whose counters give the bytes-per-count scale of FETCH_SIZE and
        # WRITE_SIZE.
        gram = torch.empty(int(db.plan.gram_off[-1]), dtype=torch.float64, device=dev)
        db.fit(precision=rp.RP_FP64, out=out)
        for _ in range(3):
            rp.rp_gram(db.plan, db.x, db.ld_x, db.y, rp.RP_FP64, gram, gram_algo=rp.RP_GRAM_MOMENTS)
        for _ in range(3):
            rp.rp_gram_jacobian(db.plan, db.x, db.ld_x, db.y, out[0], gram,
                                gram_algo=rp.RP_GRAM_MOMENTS)
        nbytes = 256 << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"probe": "gram", "copy_bytes": nbytes,
                          "gram_input_bytes": int((batch.x.shape[0] + 1) * batch.total_samples * 8),
                          "gram_output_bytes": int(db.plan.gram_off[-1]) * 8}))
        return

    if args.probe == "mfma":
        # For MFMA counter runs: three launches of each MFMA Gram of the
        # batched workload (FP64, FP32 and BF16 tiles), then the mixed forms'
        # larger-model fit kernel (4 variables, degree 4: the Gram on MFMA
        # inside k_fit) on 512 fits of 2048 samples.
        gram = torch.empty(int(db.plan.gram_off[-1]), dtype=torch.float64, device=dev)
        for prec in (rp.RP_FP64, rp.RP_MIXED_FP32, rp.RP_MIXED_BF16):
            for _ in range(3):
                rp.rp_gram(db.plan, db.x, db.ld_x, db.y, prec, gram, gram_algo=rp.RP_GRAM_MFMA)
        big = W.uniform_batch(512, 2048, 4, 4, 0.005, seed=41)
        dbb = rp.DeviceBatch(ctx, big)
        for prec in (rp.RP_MIXED_FP32, rp.RP_MIXED_BF16):
            for _ in range(2):
                dbb.fit(precision=prec)
        torch.cuda.synchronize()
        print(json.dumps({"probe": "mfma", "fits": F, "samples": args.samples,
                          "big_fits": big.num_fits, "big_samples": int(big.total_samples)}))
        return

    if args.probe == "solve":
        # For hardware-counter runs of the per-fit solver kernels: the FP64
        # fit (moment Gram + sweep + refinement), one LM step, the FP32 fit.
        for _ in range(2):
            db.fit(precision=rp.RP_FP64, out=out)
            gn_coef.copy_(out[0])
            rp.rp_refine_rational(db.plan, db.x, db.ld_x, db.y, gn_coef, gn_status, gn_loss, max_iter=1)
            db.fit(precision=rp.RP_MIXED_FP32, out=out)
        torch.cuda.synchronize()
        print(json.dumps({"probe": "solve"}))
        return

    def step(prec):
        """One step, stage by stage on the current stream, with HIP events
        between the stages (the stage breakdown)."""
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
        ev[0].record(stream)
        db.fit(precision=prec, max_refine=args.max_refine, out=out)
        ev[1].record(stream)
        coef32.copy_(out[0])
        rp.rp_loss_grad(db.plan, db.x, db.ld_x, db.y, coef32, loss32, ones, dcoef32, mode=rp.RP_LOSS_BWD)
        ev[2].record(stream)
        gn_coef.copy_(out[0])
        rp.rp_refine_rational(db.plan, db.x, db.ld_x, db.y, gn_coef, gn_status, gn_loss, max_iter=1)
        ev[3].record(stream)
        rp.rp_eval_spec_select(spec, n_t, cand_t, am, best, second)
        ev[4].record(stream)
        return ev

    side = torch.cuda.Stream()   # default priority

    def step_overlapped(prec):
        """The same step with the independent stages on a second stream: the
        program evaluation (independent of the fits) from the start, then the
        adjoint (which needs only the fitted coefficients) beside the
        Levenberg-Marquardt step; joined at the end."""
        cur = torch.cuda.current_stream()
        fork = torch.cuda.Event()
        fork.record(cur)
        side.wait_event(fork)
        with torch.cuda.stream(side):
            rp.rp_eval_spec_select(spec, n_t, cand_t, am, best, second)
        db.fit(precision=prec, max_refine=args.max_refine, out=out)
        fitted = torch.cuda.Event()
        fitted.record(cur)
        side.wait_event(fitted)
        with torch.cuda.stream(side):
            coef32.copy_(out[0])
            rp.rp_loss_grad(db.plan, db.x, db.ld_x, db.y, coef32, loss32, ones, dcoef32,
                            mode=rp.RP_LOSS_BWD)
        gn_coef.copy_(out[0])
        rp.rp_refine_rational(db.plan, db.x, db.ld_x, db.y, gn_coef, gn_status, gn_loss, max_iter=1)
        join = torch.cuda.Event()
        join.record(side)
        cur.wait_event(join)

    def outputs():
        return [t.clone() for t in (out[0], out[1], dcoef32, gn_coef, gn_loss, am, best)]

    results = {}
    for form in forms:
        prec = rp.PRECISIONS[form]
        # stage breakdown: eager steps, one stream
        for _ in range(args.warmup):
            step(prec)
        torch.cuda.synchronize()
        evs = []
        t1 = time.perf_counter()
        for _ in range(args.steps):
            evs.append(step(prec))
        torch.cuda.synchronize()
        eager_ms = 1e3 * (time.perf_counter() - t1) / args.steps
        stage = np.array([[e[i].elapsed_time(e[i + 1]) for i in range(4)] for e in evs])  # ms
        ref = outputs()
        # the step as one HIP graph (every kernel of the four stages, the
        # evaluation on its own branch), replayed: the timed form
        graph_ms, graph_ok = None, False
        if not args.no_graph:
            g = torch.cuda.CUDAGraph()
            torch.cuda.synchronize()
            with torch.cuda.graph(g):
                step_overlapped(prec)
            for _ in range(args.warmup):
                g.replay()
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            for _ in range(args.steps):
                g.replay()
            torch.cuda.synchronize()
            graph_ms = 1e3 * (time.perf_counter() - t2) / args.steps
            # every replay recomputes the same outputs from the same inputs:
            # they must equal the eager step's, bit for bit; three more
            # replays, each after eager work that overwrites the outputs, are
            # checked one by one
            graph_ok = all(bool(torch.equal(a, b)) for a, b in zip(outputs(), ref))
            for _ in range(3):
                for t in (out[0], dcoef32, gn_coef, gn_loss, best):
                    t.fill_(float("nan"))
                for t in (out[1], am):
                    t.fill_(-7)
                torch.cuda.synchronize()
                g.replay()
                torch.cuda.synchronize()
                graph_ok = graph_ok and all(bool(torch.equal(a, b)) for a, b in zip(outputs(), ref))
            if not graph_ok:
                log(form, "graph replay differs from the eager step: reporting the eager time")
        results[form] = {"wall_ms_per_step": graph_ms if graph_ok else eager_ms,
                         "eager_ms_per_step": eager_ms, "graph_ms_per_step": graph_ms,
                         "graph_matches_eager": graph_ok,
                         "stage_ms": stage.mean(axis=0).tolist(),
                         "iters_median": float(torch.median(out[3].float()).item()),
                         "status_counts": np.bincount(out[1].cpu().numpy(), minlength=6).tolist()}
        log(form, json.dumps(results[form]))

    # headline: the fastest form of the whole step; the mixed/FP64 ratio is
    # reported beside it
    head = min(forms, key=lambda f: results[f]["wall_ms_per_step"])
    ms = results[head]["wall_ms_per_step"]
    fits_per_s = F / (ms * 1e-3)
    evals = len(pw.n_grid) * int(cand_t.shape[0])
    evals_per_s = evals / (results[head]["stage_ms"][3] * 1e-3)
    mixed = [f for f in forms if f != "fp64"]
    best_mixed = min(mixed, key=lambda f: results[f]["wall_ms_per_step"]) if mixed else None

    # Roofline of the dominant kernel of the FP64 step.  Its candidates are
    # the two batched FP64 Grams by moments the step runs once each -- the
    # linear problem's (rp_gram) and the Jacobian's at the fitted coefficients
    # (rp_gram_jacobian, the LM step) -- each timed alone with HIP events on
    # the stream it runs on; the MFMA form of the linear Gram is timed beside
    # them.  Algorithmic work per launch (stated per sample):
    #   moments (k_gram_mom, FP64 VALU): one FMA per moment-weight pair,
    #     2 * moment_pairs flops -> 504 (linear) and 586 (Jacobian) for 3/3;
    #   MFMA (k_gram, FP64 MFMA): the packed upper triangle of [A b]^T [A b],
    #     (nc+1)(nc+2) flops -> 1640 for degree 3/3.
    gram = torch.empty(int(db.plan.gram_off[-1]), dtype=torch.float64, device=dev)
    db.fit(precision=rp.RP_FP64, out=out)
    fitted = out[0].clone()
    samples = float(batch.total_samples)
    nu = NC + 1
    runs = {
        "linear_moments": (lambda: rp.rp_gram(db.plan, db.x, db.ld_x, db.y, rp.RP_FP64, gram,
                                              gram_algo=rp.RP_GRAM_MOMENTS),
                           2.0 * moment_pairs(3, 3, False), "k_gram_mom_lin<3,3>"),
        "jacobian_moments": (lambda: rp.rp_gram_jacobian(db.plan, db.x, db.ld_x, db.y, fitted, gram,
                                                         gram_algo=rp.RP_GRAM_MOMENTS),
                             2.0 * moment_pairs(3, 3, True), "k_gram_mom<3,3,true>"),
        "linear_mfma": (lambda: rp.rp_gram(db.plan, db.x, db.ld_x, db.y, rp.RP_FP64, gram,
                                           gram_algo=rp.RP_GRAM_MFMA),
                        float(nu * (nu + 1)), "k_gram<3,3,fp64>"),
    }
    grams = {}
    for name, (fn, per_sample, kname) in runs.items():
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        g0, g1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = max(args.steps, 5)
        g0.record(stream)
        for _ in range(reps):
            fn()
        g1.record(stream)
        torch.cuda.synchronize()
        us = g0.elapsed_time(g1) * 1e3 / reps
        flops = samples * per_sample
        grams[name] = {"kernel": kname, "avg_launch_us": us, "flops_per_launch": flops,
                       "achieved_tflops": flops / (us * 1e-6) / 1e12,
                       "gram_equivalent_tflops": samples * nu * (nu + 1) / (us * 1e-6) / 1e12}
    log("gram", json.dumps(grams))

    # program evaluation two ways: the specialised evaluator the step runs and
    # the library's table-driven one (any program, no compile)
    am2, best2, second2 = torch.empty_like(am), torch.empty_like(best), torch.empty_like(second)
    ev_runs = {"table": lambda: rp.rp_eval_program_argmin(prog, n_t, cand_t, am2, best2, second2,
                                                          precision=rp.RP_FP64),
               "specialised": lambda: rp.rp_eval_spec_select(spec, n_t, cand_t, am, best, second)}
    ev_us = {}
    for name, fn in ev_runs.items():
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        g0, g1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = max(args.steps, 10)
        g0.record(stream)
        for _ in range(reps):
            fn()
        g1.record(stream)
        torch.cuda.synchronize()
        ev_us[name] = g0.elapsed_time(g1) * 1e3 / reps
    eval_forms = {"table_us": ev_us["table"], "specialised_us": ev_us["specialised"],
                  "specialised_compile_ms": compile_ms,
                  "evals_per_launch": evals,
                  "same_selection": bool(torch.equal(am, am2)),
                  "best_max_rel_diff": float(((best2 - best).abs() / best.abs()).max().item())}
    log("eval forms", json.dumps(eval_forms))
    dom = max(("linear_moments", "jacobian_moments"), key=lambda k: grams[k]["avg_launch_us"])
    gm = grams[dom]
    roof = {"bound": "alu", "achieved": gm["achieved_tflops"], "peak": PEAK_FP64_TFLOPS,
            "unit": "TFLOP/s", "frac": gm["achieved_tflops"] / PEAK_FP64_TFLOPS,
            "traffic": committed_traffic(gm["kernel"]),
            "kernel": gm["kernel"] + (" (FP64 Jacobian Gram by weighted moments) via rp_gram_jacobian"
                                      if dom == "jacobian_moments" else
                                      " (FP64 Gram by weighted moments) via rp_gram"),
            "avg_launch_us": gm["avg_launch_us"], "flops_per_launch": gm["flops_per_launch"],
            "others": {k: v for k, v in grams.items() if k != dom}}

    # CPU-baseline leg: the FP64 oracle on a bounded sample of the same fits,
    # timed on this host's cores; its results also give the GPU's errors.
    cpu, errs = None, {}
    if not args.no_cpu and args.cpu_sample > 0:
        import oracle
        nth = len(os.sched_getaffinity(0))
        sub = np.linspace(0, F - 1, min(args.cpu_sample, F)).astype(int)
        t2 = time.perf_counter()
        ocoef, ocoff, ostatus, _ = oracle.fit_batch(batch, nthreads=nth, fits=sub)
        dt = time.perf_counter() - t2
        cpu = {"value": len(sub) / dt, "unit": "fits/s", "cores": nth, "kind": "oracle",
               "sample": f"{len(sub)} of the {F} fits (Householder QR with pivoting, FP64), {dt:.1f} s"}
        chk = sub[np.linspace(0, len(sub) - 1, min(32, len(sub))).astype(int)]
        for form in forms:
            db.fit(precision=rp.PRECISIONS[form], max_refine=args.max_refine, out=out)
            torch.cuda.synchronize()
            c = out[0].cpu().numpy()
            worst_c, worst_p = 0.0, 0.0
            for f in chk:
                k = int(np.searchsorted(sub, f))
                a = c[db.plan.coef_off[f]:db.plan.coef_off[f + 1]]
                b = ocoef[ocoff[k]:ocoff[k + 1]]
                worst_c = max(worst_c, float(np.max(np.abs(a - b)) / np.max(np.abs(b))))
                if ostatus[k] == 0:
                    u, _ = batch.fit_samples(f)
                    pa = oracle.eval_rational(3, 3, 3, a, u)
                    pb = oracle.eval_rational(3, 3, 3, b, u)
                    worst_p = max(worst_p, float(np.max(np.abs(pa - pb)) / np.max(np.abs(pb))))
            errs[form] = {"coef_rel_err": worst_c, "pred_rel_err": worst_p, "fits_checked": len(chk)}
        # selection agreement of the program evaluation on 64 of the data sizes
        rp.rp_eval_spec_select(spec, n_t, cand_t, am, best, second)
        torch.cuda.synchronize()
        coefs = [rp.planted_coefs(mm) for mm in pw.metrics]
        off = np.zeros(len(coefs) + 1, dtype=np.int64)
        np.cumsum([len(cc) for cc in coefs], out=off[1:])
        deg = np.array([mm.deg_num for mm in pw.metrics], dtype=np.int32)
        oprog = oracle.Program(oracle.TEMPLATE_MWPCWP, 3, deg, deg, np.concatenate(coefs), off,
                               hw=pw.hw, hw_stride=17, scale=pw.scales)
        jj = np.linspace(0, len(pw.n_grid) - 1, 64).astype(int)
        cands = cand_t.cpu().numpy()
        t3 = time.perf_counter()
        oam, obest, osec = oracle.argmin(oprog, pw.n_grid[jj], cands)
        dt3 = time.perf_counter() - t3
        gam = am.cpu().numpy()[0, jj]
        gbest = best.cpu().numpy()[0, jj]
        agree = int(np.sum(gam == oam[0]))
        ties = int(np.sum((gam != oam[0]) & (osec[0] <= obest[0] * (1 + 1e-6))))
        errs["eval_argmin"] = {"n_checked": len(jj), "same_index": agree, "within_tie_window": ties,
                               "best_rel_err": float(np.max(np.abs(gbest - obest[0]) / obest[0]))}
        cpu["evals_per_s"] = len(jj) * len(cands) / dt3
        log("errors", json.dumps(errs))

    line = {
        "metric": "rational fits/s + candidate evals/s, mixed-precision batched vs plain FP64",
        "value": fits_per_s, "unit": "fits/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": {"fp32": "f32+f64", "bf16": "bf16+f64", "fp64": "f64"}[head],
        "data": "synthetic",
        "config": {"workload": f"batched fit {F} fits x {args.samples} samples, v=3, degree 3/3 "
                               "(fit + adjoint + one LM step) and MWP-CWP program over 1024 data "
                               "sizes x 230 block formats (evaluation + argmin, specialised "
                               "evaluator compiled at set-up)",
                   "form": head},
        "evals_per_s": evals_per_s,
        "eval_forms": eval_forms,
        "forms": {k: {"ms_per_step": v["wall_ms_per_step"],
                      "eager_ms_per_step": v["eager_ms_per_step"],
                      "graph_ms_per_step": v["graph_ms_per_step"],
                      "graph_matches_eager": v["graph_matches_eager"],
                      "fits_per_s": F / (v["wall_ms_per_step"] * 1e-3),
                      "stages_ms": dict(zip(["fit", "adjoint", "lm_step", "eval_argmin"], v["stage_ms"])),
                      "refine_iters_median": v["iters_median"]}
                  for k, v in results.items()},
        "mixed_vs_fp64": (results["fp64"]["wall_ms_per_step"] / results[best_mixed]["wall_ms_per_step"]
                          if best_mixed and "fp64" in results else None),
        "errors_vs_oracle": errs,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
