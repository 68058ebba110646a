"""Every fit of the two large workloads against the FP64 oracle, in all three
arithmetic forms: the batched workload (4096 fits x 2048 samples, three
variables, degree 3/3) and the uneven one (16384 fits, m log-uniform in
[64, 8192], v in {2, 3, 4}, degree 1..4).

Bars (one per kind of result):
  * status: equal on every fit.  The one decision both sides take from
    floating point near a boundary is "Q <= 0 at some sample" (status 4 vs 0):
    the GPU takes min Q at coefficients that differ from the oracle's by
    rounding, so a fit whose oracle min Q lies within QWIN of zero may differ;
    such fits are counted and printed (none occur in these workloads).  The
    mixed forms never flag rank deficiency (their shifted factorisation keeps
    every pivot); a fit the oracle calls rank deficient is compared by
    predictions there (none occur either).
  * FP64 form: coefficients within 1e-9 relative (max norm) on every fit,
    minimum-norm solutions of underdetermined fits included.
  * mixed forms, every full-rank fit (oracle status 0 or 4): predictions N/Q
    within 1e-6 relative over the samples where the oracle's |Q| >= 1e-3
    (near a root of Q the prediction is unbounded and says nothing about the
    fit), and coefficients within 1e-6 relative (max norm), which holds at
    every sample; underdetermined fits: the FP64 minimum-norm re-solve, 1e-9.
"""
import sys

import numpy as np
import pytest

from paper_1906_00142_amd import rp
from paper_1906_00142_amd import workloads as W
from tests._parity import masked_pred_rel_err, q_values

pytestmark = pytest.mark.gpu

COEF_TOL = 1e-9
MIXED_COEF_TOL = 1e-6
PRED_TOL = 1e-6
QWIN = 1e-8


def say(*a):
    print(*a, file=sys.stderr, flush=True)


class Workload:
    def __init__(self, name, batch):
        self.name, self.batch = name, batch
        self.gpu = {}
        self.iters = {}
        self.oracle = None


def _run(gpu_ctx, orc, name, batch):
    import torch
    w = Workload(name, batch)
    db = rp.DeviceBatch(gpu_ctx, batch)
    w.coff = np.asarray(db.plan.coef_off)
    for form in ("fp64", "fp32", "bf16"):
        say(name, "fit", form)
        coef, status, resid, iters = db.fit(precision=rp.PRECISIONS[form])
        torch.cuda.synchronize()
        w.gpu[form] = (coef.cpu().numpy(), status.cpu().numpy())
        w.iters[form] = iters.cpu().numpy()
    # the tuned per-bucket form: eager, and as a graph replayed with eager
    # work between the replays
    say(name, "tune")
    rp.rp_plan_tune(db.plan, db.x, db.ld_x, db.y)
    w.tuning = rp.rp_plan_tuning(db.plan)
    say(name, "tuning table", rp.TUNE_COLUMNS, w.tuning.tolist())
    coef, status, resid, iters = db.fit(precision=rp.RP_AUTO)
    torch.cuda.synchronize()
    w.gpu["auto"] = (coef.cpu().numpy(), status.cpu().numpy())
    out = db.alloc_fit_outputs()
    g = rp.FitGraph(db, *out, precision=rp.RP_AUTO)
    w.graph_equal = []
    for rep in range(2):
        for t in out:
            t.zero_()
        g.launch()
        torch.cuda.synchronize()
        torch.randn(1000, device=db.device).sum().item()
        w.graph_equal.append(bool(torch.equal(out[0], coef) and torch.equal(out[1], status)))
    g.close()
    say(name, "oracle on", batch.num_fits, "fits")
    oc, ocoff, ost, ores = orc.fit_batch(batch, nthreads=16)
    assert np.array_equal(ocoff, w.coff)
    w.oracle = (oc, ost)
    # the oracle's min Q per fit, for the status window
    w.qmin = np.empty(batch.num_fits)
    for f in range(batch.num_fits):
        u, _ = batch.fit_samples(f)
        v, d = int(batch.nvars[f]), int(batch.deg_num[f])
        q = q_values(orc, u, oc[w.coff[f]:w.coff[f + 1]], v, d, d) if u.shape[1] else np.ones(1)
        w.qmin[f] = q.min()
    del db
    torch.cuda.empty_cache()
    return w


@pytest.fixture(scope="module")
def batched(gpu_ctx, orc):
    return _run(gpu_ctx, orc, "batched", W.batched_fit())


@pytest.fixture(scope="module")
def uneven(gpu_ctx, orc):
    return _run(gpu_ctx, orc, "uneven", W.uneven_batch())


def check_statuses(w, form):
    st = w.gpu[form][1]
    ost = w.oracle[1]
    diff = np.where(st != ost)[0]
    explained = [f for f in diff
                 if {int(st[f]), int(ost[f])} == {0, 4} and abs(w.qmin[f]) <= QWIN]
    if form != "fp64":
        explained += [f for f in diff if ost[f] == 1 and st[f] in (0, 4)]
    say(w.name, form, "status counts gpu", np.bincount(st, minlength=6).tolist(),
        "oracle", np.bincount(ost, minlength=6).tolist(),
        "disagreements", len(diff), "within the stated windows", len(explained))
    unexplained = sorted(set(diff.tolist()) - set(explained))
    assert not unexplained, [(f, int(st[f]), int(ost[f]), float(w.qmin[f])) for f in unexplained[:10]]
    return len(diff)


def check_fp64(w):
    c, st = w.gpu["fp64"]
    oc, ost = w.oracle
    check_statuses(w, "fp64")
    worst, wf = 0.0, -1
    for f in range(w.batch.num_fits):
        a, o = c[w.coff[f]:w.coff[f + 1]], oc[w.coff[f]:w.coff[f + 1]]
        if len(o) == 0 or ost[f] == 3:
            continue
        e = np.max(np.abs(a - o)) / np.max(np.abs(o))
        if e > worst:
            worst, wf = e, f
    say(w.name, "fp64 worst coefficient error", worst, "fit", wf, "over", w.batch.num_fits, "fits")
    assert worst <= COEF_TOL, (wf, worst)


def check_mixed(orc, w, form):
    c, st = w.gpu[form]
    oc, ost = w.oracle
    check_statuses(w, form)
    b = w.batch
    worst_p = worst_c = worst_u = 0.0
    n_full = n_under = 0
    bad = []
    for f in range(b.num_fits):
        a, o = c[w.coff[f]:w.coff[f + 1]], oc[w.coff[f]:w.coff[f + 1]]
        if ost[f] in (0, 1, 4):
            u, _ = b.fit_samples(f)
            v, d = int(b.nvars[f]), int(b.deg_num[f])
            ep = masked_pred_rel_err(orc, u, v, d, d, a, o)
            worst_p = max(worst_p, ep)
            ec = np.max(np.abs(a - o)) / np.max(np.abs(o)) if ost[f] != 1 else 0.0
            worst_c = max(worst_c, ec)
            if ep > PRED_TOL or ec > MIXED_COEF_TOL:
                bad.append((f, v, d, int(st[f]), int(w.iters[form][f]), ep, ec))
            n_full += 1
        elif ost[f] == 2:
            eu = np.max(np.abs(a - o)) / np.max(np.abs(o))
            worst_u = max(worst_u, eu)
            if eu > COEF_TOL:
                bad.append((f, int(b.nvars[f]), int(b.deg_num[f]), int(st[f]), int(w.iters[form][f]), eu, eu))
            n_under += 1
    say(w.name, form, "full-rank fits", n_full, "worst prediction error", worst_p,
        "worst coefficient error", worst_c, "; underdetermined fits", n_under,
        "worst coefficient error", worst_u)
    assert not bad, ("fits beyond the bars (fit, v, d, status, iters, pred err, coef err)",
                     len(bad), bad[:10])


def test_batched_fp64_every_fit(batched):
    check_fp64(batched)


@pytest.mark.parametrize("form", ["fp32", "bf16"])
def test_batched_mixed_every_fit(orc, batched, form):
    check_mixed(orc, batched, form)


def test_uneven_fp64_every_fit(uneven):
    check_fp64(uneven)
    assert np.sum(uneven.gpu["fp64"][1] == rp.RP_FIT_NOT_CONVERGED) == 0


@pytest.mark.parametrize("form", ["fp32", "bf16"])
def test_uneven_mixed_every_fit(orc, uneven, form):
    check_mixed(orc, uneven, form)
    assert np.sum(uneven.gpu[form][1] == rp.RP_FIT_NOT_CONVERGED) == 0


@pytest.mark.parametrize("wl", ["batched", "uneven"])
def test_tuned_form_every_fit(request, wl):
    """RP_AUTO: every bucket in the form the tuner measured fastest.  Its
    results equal that form's run bit for bit (same kernels, same inputs),
    the graph replays equal the eager run, and so every fit meets the chosen
    form's bar against the oracle (checked above)."""
    w = request.getfixturevalue(wl)
    assert all(w.graph_equal), w.graph_equal
    names = {rp.RP_FP64: "fp64", rp.RP_MIXED_FP32: "fp32", rp.RP_MIXED_BF16: "bf16"}
    chosen = {(int(r[0]), int(r[1])): (names[int(r[3])], int(r[4])) for r in w.tuning}
    c, st = w.gpu["auto"]
    b = w.batch
    counts = {}
    for f in range(b.num_fits):
        form, algo = chosen[(int(b.nvars[f]), int(b.deg_num[f]))]
        counts[form] = counts.get(form, 0) + 1
        if form == "fp64" and algo != rp.RP_GRAM_MOMENTS:
            # the FP64 run above formed its Gram by moments: here the oracle
            oc, ost = w.oracle
            a, o = c[w.coff[f]:w.coff[f + 1]], oc[w.coff[f]:w.coff[f + 1]]
            assert st[f] == ost[f] or ({int(st[f]), int(ost[f])} == {0, 4} and abs(w.qmin[f]) <= QWIN)
            if len(o) and ost[f] != 3:
                assert np.max(np.abs(a - o)) <= COEF_TOL * np.max(np.abs(o)), f
            continue
        rc, rst = w.gpu[form]
        assert st[f] == rst[f]
        assert np.array_equal(c[w.coff[f]:w.coff[f + 1]], rc[w.coff[f]:w.coff[f + 1]]), f
    say(wl, "tuned forms per fit", counts)
