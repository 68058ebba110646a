"""The uneven workload at full size: 16384 fits, m log-uniform in [64, 8192],
v in {2, 3, 4}, d in {1, 2, 3, 4}; then every fitted model is evaluated over
4096 candidates at 4 data sizes with an argmin per data size; the oracle
checks the selections of programs spread over each shape bucket."""
import sys

import numpy as np
import pytest

from paper_1906_00142_amd import rp
from paper_1906_00142_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def uneven():
    b = W.uneven_batch()
    say("uneven workload", b.num_fits, "fits,", b.total_samples, "samples")
    return b


def candidate_grid(v):
    """4096 program-parameter candidates for a model in v variables: a 1-D grid
    of 4096 points (v = 2), 64 x 64 (v = 3) or 16^3 (v = 4), in 1..G per axis."""
    g = {2: 4096, 3: 64, 4: 16}[v]
    axes = [np.arange(1, g + 1)] * (v - 1)
    mesh = np.meshgrid(*axes, indexing="ij")
    cand = np.stack([a.ravel() for a in mesh], axis=-1).astype(np.int32)
    return cand, [4096.0] + [float(g)] * (v - 1)


def test_uneven_fit_and_select(gpu_ctx, orc, uneven):
    import torch
    b = uneven
    db = rp.DeviceBatch(gpu_ctx, b)
    coef, status, resid, iters = db.fit()
    torch.cuda.synchronize()
    c = coef.cpu().numpy()
    st = status.cpu().numpy()
    coff = db.plan.coef_off
    say("status counts", np.bincount(st, minlength=6).tolist())
    # (every fit's coefficients and status: tests/test_gpu_full_parity.py)

    # selection: every fitted model of one shape bucket is a program
    n_grid = np.array([1024.0, 2048.0, 3072.0, 4096.0])
    dev = db.device
    for v in (2, 3, 4):
        for d in (2, 4):
            idx = np.where((b.nvars == v) & (b.deg_num == d) & (st == 0))[0]
            if len(idx) == 0:
                continue
            coefs = [c[coff[f]:coff[f + 1]] for f in idx]
            off = np.zeros(len(idx) + 1, np.int64)
            np.cumsum([len(x) for x in coefs], out=off[1:])
            deg = np.full(len(idx), d, np.int32)
            cand, scale = candidate_grid(v)
            coef_t = torch.from_numpy(np.concatenate(coefs)).to(dev)
            prog = rp.Program(gpu_ctx, rp.RP_TEMPLATE_SINGLE, v, deg, deg, off, coef_t, scale,
                              num_programs=len(idx))
            P = len(idx)
            am = torch.empty((P, 4), dtype=torch.int32, device=dev)
            best = torch.empty((P, 4), dtype=torch.float64, device=dev)
            second = torch.empty((P, 4), dtype=torch.float64, device=dev)
            rp.rp_eval_program_argmin(prog, torch.from_numpy(n_grid).to(dev),
                                      torch.from_numpy(cand).to(dev), am, best, second)
            torch.cuda.synchronize()
            am, best = am.cpu().numpy(), best.cpu().numpy()
            sub = np.linspace(0, P - 1, min(5, P)).astype(int)
            oprog = orc.Program(orc.TEMPLATE_SINGLE, v, deg[sub], deg[sub],
                                np.concatenate([coefs[i] for i in sub]),
                                np.concatenate([[0], np.cumsum([len(coefs[i]) for i in sub])]),
                                scale=scale, num_programs=len(sub))
            oam, obest, osec = orc.argmin(oprog, n_grid, cand)
            for k, p in enumerate(sub):
                for j in range(4):
                    if am[p, j] != oam[k, j]:
                        assert osec[k, j] <= obest[k, j] * (1 + 1e-6) or \
                            abs(oprog.value(k, n_grid[j], cand[am[p, j]]) - obest[k, j]) <= 1e-6 * abs(obest[k, j])
                    np.testing.assert_allclose(best[p, j], obest[k, j], rtol=1e-9)
            say("selection checked", v, d, "programs", P)


def test_graph_replays_match_eager_and_tuning_roundtrip(gpu_ctx, tmp_path):
    """The captured fit graph, replayed several times with eager work in
    between, gives the eager result every time; the tuning table survives a
    save/load round trip and the tuned plan still fits identically."""
    import torch
    b = W.uneven_batch(num_fits=300, m_lo=64, m_hi=3000, seed=9)
    db = rp.DeviceBatch(gpu_ctx, b)
    ref = db.fit()
    torch.cuda.synchronize()
    ref = [t.clone() for t in ref]
    out = db.alloc_fit_outputs()
    g = rp.FitGraph(db, *out)
    for rep in range(3):
        for t in out:
            t.zero_()
        g.launch()
        torch.cuda.synchronize()
        junk = torch.randn(1000, device=db.device).sum().item()   # eager work between replays
        for a_, b_ in zip(out, ref):
            assert torch.equal(a_, b_), rep
    g.close()
    rp.rp_plan_tune(db.plan, db.x, db.ld_x, db.y)
    t = rp.rp_plan_tuning(db.plan)
    say("tuning table", rp.TUNE_COLUMNS, t.tolist())
    assert len(t) >= 4 and set(t[:, 4].tolist()) <= {rp.RP_GRAM_MFMA, rp.RP_GRAM_MOMENTS}
    assert set(t[:, 3].tolist()) <= {rp.RP_FP64, rp.RP_MIXED_FP32, rp.RP_MIXED_BF16}
    assert np.all(t[:, 5:] > 0)
    # the chosen form is the fastest measured one
    best = np.argmin(t[:, 5:], axis=1)
    assert np.array_equal(t[:, 3], np.array([rp.RP_FP64, rp.RP_FP64, rp.RP_MIXED_FP32,
                                             rp.RP_MIXED_BF16])[best])
    path = str(tmp_path / "tune.json")
    rp.save_tuning(db.plan, path)
    db2 = rp.DeviceBatch(gpu_ctx, b)
    rp.load_tuning(db2.plan, path)
    np.testing.assert_array_equal(rp.rp_plan_tuning(db2.plan), t)
    c2 = db2.fit()[0]
    torch.cuda.synchronize()
    st = ref[1].cpu().numpy()
    c_ref, c_new = ref[0].cpu().numpy(), c2.cpu().numpy()
    for f in range(b.num_fits):
        if st[f] in (0, 4):
            a_, o_ = c_new[db.plan.coef_off[f]:db.plan.coef_off[f + 1]], c_ref[db.plan.coef_off[f]:db.plan.coef_off[f + 1]]
            assert np.max(np.abs(a_ - o_)) <= 1e-9 * np.max(np.abs(o_))
