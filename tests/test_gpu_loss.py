"""GPU parity of the true-loss path: the FP32 adjoint kernel behind a
torch.autograd.Function and the FP64 Levenberg-Marquardt refinement.

Bars: FP32 loss within 1e-4 relative of the oracle's FP64 loss; FP32 gradient
within 1e-3 of max|grad| of the oracle's closed-form gradient, which is itself
checked against central differences (h = 1e-6, FP64) here; refinement: final
loss within 1e-9 relative and coefficients within 1e-6 relative of the
oracle's LM result from the same start.
"""
import sys

import numpy as np
import pytest

from paper_1906_00142_amd import rp
from paper_1906_00142_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def start_coefs(orc, batch):
    coef, coff, status, _ = orc.fit_batch(batch, nthreads=8)
    return coef, coff, status


def test_loss_and_adjoint_against_oracle(gpu_ctx, orc):
    import torch
    v, d = 3, 3
    batch = W.uniform_batch(12, 2048, v, d, 0.005, seed=61)
    coef, coff, status = start_coefs(orc, batch)
    db = rp.DeviceBatch(gpu_ctx, batch)
    c32 = torch.from_numpy(coef.astype(np.float32)).to(db.device)
    loss = torch.empty(batch.num_fits, dtype=torch.float32, device=db.device)
    dloss = torch.linspace(0.5, 2.0, batch.num_fits, dtype=torch.float32, device=db.device)
    dcoef = torch.empty_like(c32)
    rp.rp_loss_grad(db.plan, db.x, db.ld_x, db.y, c32, loss, dloss, dcoef, mode=rp.RP_LOSS_BWD)
    torch.cuda.synchronize()
    L = loss.cpu().numpy()
    G = dcoef.cpu().numpy()
    w = dloss.cpu().numpy()
    for f in range(batch.num_fits):
        if status[f] != 0:
            continue
        u, y = batch.fit_samples(f)
        c = coef[coff[f]:coff[f + 1]].astype(np.float32).astype(np.float64)
        oL, og = orc.loss_grad(u, y, d, d, c)
        np.testing.assert_allclose(L[f], oL, rtol=1e-4)
        gg = G[coff[f]:coff[f + 1]] / w[f]
        assert np.max(np.abs(gg - og)) <= 1e-3 * np.max(np.abs(og)), f
        # central differences of the FP64 loss on two coordinates
        for k in (0, len(c) - 1):
            h = 1e-6
            cp, cm = c.copy(), c.copy()
            cp[k] += h
            cm[k] -= h
            fd = (orc.loss_grad(u, y, d, d, cp)[0] - orc.loss_grad(u, y, d, d, cm)[0]) / (2 * h)
            assert abs(fd - og[k]) <= 1e-6 * max(abs(og[k]), 1e-12 * np.max(np.abs(og))) + 1e-9 * np.max(np.abs(og))


@pytest.mark.parametrize("v,d,nfit,m", [(3, 4, 4, 700), (4, 4, 2, 300), (1, 2, 6, 77), (2, 3, 5, 130)])
def test_loss_and_adjoint_shapes_at_planted(gpu_ctx, orc, v, d, nfit, m):
    """Loss and gradient at the planted coefficients (denominators bounded away
    from zero) for shapes with fewer and with more unknowns than a wave has
    lanes, and ragged sample counts."""
    import torch
    from conftest import planted_in_order
    batch = W.uniform_batch(nfit, m, v, d, 0.005, seed=71 + 10 * v + d)
    db = rp.DeviceBatch(gpu_ctx, batch)
    coff = db.plan.coef_off
    coef = np.concatenate([planted_in_order(orc, batch.planted[f]) for f in range(nfit)])
    assert len(coef) == coff[-1]
    c32 = torch.from_numpy(coef.astype(np.float32)).to(db.device)
    loss = torch.empty(nfit, dtype=torch.float32, device=db.device)
    dloss = torch.linspace(0.5, 2.0, nfit, dtype=torch.float32, device=db.device)
    dcoef = torch.empty_like(c32)
    rp.rp_loss_grad(db.plan, db.x, db.ld_x, db.y, c32, loss, dloss, dcoef, mode=rp.RP_LOSS_BWD)
    torch.cuda.synchronize()
    L, G, w = loss.cpu().numpy(), dcoef.cpu().numpy(), dloss.cpu().numpy()
    for f in range(nfit):
        u, y = batch.fit_samples(f)
        c = coef[coff[f]:coff[f + 1]].astype(np.float32).astype(np.float64)
        oL, og = orc.loss_grad(u, y, d, d, c)
        np.testing.assert_allclose(L[f], oL, rtol=1e-4)
        gg = G[coff[f]:coff[f + 1]] / w[f]
        assert np.max(np.abs(gg - og)) <= 1e-3 * np.max(np.abs(og)), f


def test_autograd_function_matches_backward_entry(gpu_ctx, orc):
    import torch
    batch = W.uniform_batch(6, 500, 2, 2, 0.01, seed=62)
    coef, coff, status = start_coefs(orc, batch)
    db = rp.DeviceBatch(gpu_ctx, batch)
    Fn = rp.rational_loss_function()
    c = torch.from_numpy(coef.astype(np.float32)).to(db.device).requires_grad_(True)
    loss = Fn.apply(c, db)
    wts = torch.arange(1, batch.num_fits + 1, dtype=torch.float32, device=db.device)
    (loss * wts).sum().backward()
    ref = torch.empty_like(c)
    l2 = torch.empty_like(loss)
    rp.rp_loss_grad(db.plan, db.x, db.ld_x, db.y, c.detach(), l2, wts, ref, mode=rp.RP_LOSS_BWD)
    torch.cuda.synchronize()
    torch.testing.assert_close(c.grad, ref, rtol=0, atol=0)
    torch.testing.assert_close(loss.detach(), l2, rtol=0, atol=0)


def test_adam_then_fp64_gauss_newton(gpu_ctx, orc):
    """Adam on the FP32 adjoint, then FP64 LM steps; LM result matches the oracle's."""
    import torch
    batch = W.uniform_batch(16, 1024, 3, 2, 0.005, seed=63)
    coef, coff, status = start_coefs(orc, batch)
    db = rp.DeviceBatch(gpu_ctx, batch)
    Fn = rp.rational_loss_function()
    c = torch.from_numpy(coef.astype(np.float32)).to(db.device).requires_grad_(True)
    opt = torch.optim.Adam([c], lr=1e-4)
    l0 = Fn.apply(c, db).detach().clone()
    for _ in range(20):
        opt.zero_grad()
        Fn.apply(c, db).sum().backward()
        opt.step()
    l1 = Fn.apply(c, db).detach()
    start = c.detach().to(torch.float64).contiguous()
    st = torch.zeros(batch.num_fits, dtype=torch.int32, device=db.device)
    loss = torch.zeros(batch.num_fits, dtype=torch.float64, device=db.device)
    rp.rp_refine_rational(db.plan, db.x, db.ld_x, db.y, start, st, loss, max_iter=50, rtol=1e-14)
    torch.cuda.synchronize()
    s = start.cpu().numpy()
    Lg = loss.cpu().numpy()
    stg = st.cpu().numpy()
    c0 = c.detach().to(torch.float64).cpu().numpy()
    ok = 0
    for f in range(batch.num_fits):
        if status[f] != 0:
            continue
        u, y = batch.fit_samples(f)
        oc, oL, oit = orc.refine(u, y, 2, 2, c0[coff[f]:coff[f + 1]], max_iter=50, rtol=1e-14)
        np.testing.assert_allclose(Lg[f], oL, rtol=1e-9)
        assert np.max(np.abs(s[coff[f]:coff[f + 1]] - oc)) <= 1e-6 * np.max(np.abs(oc))
        assert stg[f] == 0
        ok += 1
    say("refined fits", ok, "adam loss change", float((l1 - l0).sum()))
    assert ok >= 4


def test_differentiation_workload_full_size(gpu_ctx, orc):
    """4096 fits x 2048 samples, degree 3/3: 200 Adam iterations on the FP32
    adjoint from the linearised fits, then FP64 Levenberg-Marquardt steps; the
    oracle's LM from the same Adam end point checks a sample of fits."""
    import torch
    batch = W.refine_batch()
    db = rp.DeviceBatch(gpu_ctx, batch)
    coef, status, resid, iters = db.fit()
    torch.cuda.synchronize()
    st0 = status.cpu().numpy()
    Fn = rp.rational_loss_function()
    c = coef.to(torch.float32).clone().requires_grad_(True)
    opt = torch.optim.Adam([c], lr=1e-5)
    l0 = Fn.apply(c, db).detach().clone()
    for _ in range(200):
        opt.zero_grad()
        Fn.apply(c, db).sum().backward()
        opt.step()
    l1 = Fn.apply(c, db).detach()
    ok = (st0 == 0).nonzero()[0]
    okt = torch.from_numpy(ok).to(db.device)
    say("adam: loss sum over OK fits", float(l0[okt].sum()), "->", float(l1[okt].sum()))
    start = c.detach().to(torch.float64).contiguous()
    c0 = start.cpu().numpy().copy()
    st = torch.zeros(batch.num_fits, dtype=torch.int32, device=db.device)
    loss = torch.zeros(batch.num_fits, dtype=torch.float64, device=db.device)
    rp.rp_refine_rational(db.plan, db.x, db.ld_x, db.y, start, st, loss, max_iter=30)
    torch.cuda.synchronize()
    s, L, stg = start.cpu().numpy(), loss.cpu().numpy(), st.cpu().numpy()
    coff = db.plan.coef_off
    pick = ok[np.linspace(0, len(ok) - 1, 12).astype(int)]
    for f in pick:
        u, y = batch.fit_samples(f)
        oc, oL, oit = orc.refine(u, y, 3, 3, c0[coff[f]:coff[f + 1]], max_iter=30, rtol=1e-14)
        np.testing.assert_allclose(L[f], oL, rtol=1e-9)
        assert np.max(np.abs(s[coff[f]:coff[f + 1]] - oc)) <= 1e-6 * np.max(np.abs(oc))
    say("LM status counts", np.bincount(stg, minlength=6).tolist())
