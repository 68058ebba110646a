"""GPU parity of the minimum-norm solutions (Section 4.2 solves each fit with
an SVD, whose answer on a rank-deficient or underdetermined system is the
least-squares minimiser of smallest norm) against the oracle's complete
orthogonal decomposition.

Bars: coefficient vector relative error (max-norm) <= 1e-9 and identical
status codes, for fits with fewer samples than unknowns in general position,
fits whose samples repeat (dependent rows), and fits whose design loses rank
through collinear or few-valued variables.
"""
import sys

import numpy as np
import pytest

from paper_1906_00142_amd import rp
from paper_1906_00142_amd import workloads as W

pytestmark = pytest.mark.gpu

COEF_TOL = 1e-9
SHAPES = [(1, 2), (1, 4), (2, 2), (2, 4), (3, 2), (3, 3), (3, 4), (4, 2), (4, 3), (4, 4)]


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def make_batch(parts):
    """FitBatch from (u [v x m], y [m], v, d) parts; u padded to 4 rows."""
    off = np.zeros(len(parts) + 1, dtype=np.int64)
    np.cumsum([len(p[1]) for p in parts], out=off[1:])
    x = np.zeros((4, max(int(off[-1]), 1)))
    for p, a in zip(parts, off[:-1]):
        x[:p[2], a:a + len(p[1])] = p[0]
    ys = np.concatenate([p[1] for p in parts]) if off[-1] else np.zeros(1)
    nv = np.array([p[2] for p in parts], np.int32)
    dg = np.array([p[3] for p in parts], np.int32)
    return W.FitBatch(len(parts), 4, off, nv, dg, dg.copy(), x, ys, 0.005)


def planted_samples(rng, v, d, m):
    pl = W.plant(rng, v, d, d)
    u = rng.uniform(0.0, 1.0, size=(v, m))
    y = pl.value(u) * (1.0 + 0.005 * rng.normal(size=m))
    return u, y


def fit_and_compare(ctx, orc, batch, precision=rp.RP_FP64, label=""):
    import torch
    db = rp.DeviceBatch(ctx, batch)
    coef, status, resid, iters = db.fit(precision=precision)
    torch.cuda.synchronize()
    coef, status, resid = coef.cpu().numpy(), status.cpu().numpy(), resid.cpu().numpy()
    coff = db.plan.coef_off
    ocoef, ocoff, ostatus, oresid = orc.fit_batch(batch, nthreads=8)
    worst = 0.0
    for f in range(batch.num_fits):
        a, b = coef[coff[f]:coff[f + 1]], ocoef[coff[f]:coff[f + 1]]
        e = np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)
        worst = max(worst, e)
        m = int(batch.sample_off[f + 1] - batch.sample_off[f])
        case = (label, f, int(batch.nvars[f]), int(batch.deg_num[f]), m)
        assert status[f] == ostatus[f], (case, status[f], ostatus[f])
        assert e <= COEF_TOL, (case, e)
        scale = max(np.linalg.norm(batch.fit_samples(f)[1]), 1e-300)
        assert abs(resid[f] - oresid[f]) <= 1e-9 * scale, (case, resid[f], oresid[f])
    say(label, "fits", batch.num_fits, "worst coefficient error", worst)
    return status


@pytest.mark.parametrize("precision", [rp.RP_FP64, rp.RP_MIXED_FP32, rp.RP_MIXED_BF16])
def test_underdetermined_general_position(gpu_ctx, orc, precision):
    rng = np.random.default_rng(2024)
    parts = []
    for v, d in SHAPES:
        nc = orc.num_coefs(v, d, d)
        for m in sorted({1, 2, nc // 2, nc - 2, nc - 1}):
            u, y = planted_samples(rng, v, d, m)
            parts.append((u, y, v, d))
    st = fit_and_compare(gpu_ctx, orc, make_batch(parts), precision, f"underdetermined/{precision}")
    assert np.all(st == rp.RP_FIT_UNDERDETERMINED)


def test_underdetermined_with_repeated_samples(gpu_ctx, orc):
    """Repeated samples make the sample Gram singular (dependent rows): the
    unknown-space form takes over."""
    rng = np.random.default_rng(7)
    parts = []
    for v, d, mu, rep in [(1, 4, 3, 2), (2, 2, 8, 2), (2, 3, 12, 3), (3, 2, 6, 3), (3, 4, 40, 10),
                          (4, 4, 60, 20)]:
        u, y = planted_samples(rng, v, d, mu)
        parts.append((np.concatenate([u, u[:, :rep]], axis=1), np.concatenate([y, y[:rep]]), v, d))
    st = fit_and_compare(gpu_ctx, orc, make_batch(parts), rp.RP_FP64, "repeated samples")
    assert np.all(st == rp.RP_FIT_UNDERDETERMINED)


def test_rank_deficient_designs(gpu_ctx, orc):
    """m >= unknowns, rank lost through the sample design: equal variables,
    variables that take two or three values, a constant variable."""
    rng = np.random.default_rng(11)
    parts = []
    t = rng.uniform(0, 1, 60)
    parts.append((np.stack([t, t]), 1.0 + 0.5 * t + 0.01 * rng.normal(size=60), 2, 2))
    t = rng.uniform(0, 1, 300)
    parts.append((np.stack([t, t]), (1.0 + t) / (1 + 0.1 * t) * (1 + 0.005 * rng.normal(size=300)), 2, 3))
    a, b2 = rng.uniform(0, 1, 200), rng.choice([0.25, 0.75], 200)
    parts.append((np.stack([a, b2]), (1 + a * b2) * (1 + 0.005 * rng.normal(size=200)), 2, 3))
    a, b3, c3 = rng.uniform(0, 1, 400), rng.choice([0.25, 0.5, 1.0], 400), rng.uniform(0, 1, 400)
    parts.append((np.stack([a, b3, c3]), (1 + a * b3 + c3) * (1 + 0.005 * rng.normal(size=400)), 3, 4))
    t, s = rng.uniform(0, 1, 500), rng.uniform(0, 1, 500)
    parts.append((np.stack([t, s, t]), 1.0 + t + 0.01 * rng.normal(size=500), 3, 3))
    u = rng.uniform(0, 1, (4, 900))
    u[3] = 0.5
    parts.append((u, (1 + u[0] * u[1] + u[2]) * (1 + 0.005 * rng.normal(size=900)), 4, 4))
    u = rng.uniform(0, 1, (4, 300))
    u[1] = u[0]
    parts.append((u, (1 + u[0] + u[2] * u[3]) * (1 + 0.005 * rng.normal(size=300)), 4, 2))
    st = fit_and_compare(gpu_ctx, orc, make_batch(parts), rp.RP_FP64, "rank deficient")
    assert np.all(st == rp.RP_FIT_RANK_DEFICIENT)


def test_min_norm_is_deterministic_over_many_fits(gpu_ctx, orc):
    """Two fits of the same batch give identical bits; flagged fits are
    scattered over the bucket so several workgroups serve several fits."""
    import torch
    rng = np.random.default_rng(5)
    parts = []
    for k in range(600):
        v, d = 4, 4
        m = 80 + (k * 37) % 140          # about half of them below 139 unknowns
        u, y = planted_samples(rng, v, d, m)
        parts.append((u, y, v, d))
    batch = make_batch(parts)
    db = rp.DeviceBatch(gpu_ctx, batch)
    c1, s1, r1, _ = [t.clone() for t in db.fit()]
    c2, s2, r2, _ = [t.clone() for t in db.fit()]
    torch.cuda.synchronize()
    assert torch.equal(c1, c2) and torch.equal(s1, s2)
    st = s1.cpu().numpy()
    under = np.where(st == rp.RP_FIT_UNDERDETERMINED)[0]
    say("underdetermined", len(under), "of", batch.num_fits)
    assert len(under) > 200
    pick = under[np.linspace(0, len(under) - 1, 12).astype(int)]
    ocoef, ocoff, ost, ores = orc.fit_batch(batch, nthreads=8, fits=pick)
    c = c1.cpu().numpy()
    for k, f in enumerate(pick):
        a, b = c[db.plan.coef_off[f]:db.plan.coef_off[f + 1]], ocoef[ocoff[k]:ocoff[k + 1]]
        assert np.max(np.abs(a - b)) / np.max(np.abs(b)) <= COEF_TOL, f


def test_unknown_space_form_several_fits_per_workgroup(gpu_ctx, orc):
    """More rank-deficient fits than the re-solve pass has workgroups (256),
    so each workgroup solves two or three in a row in the unknown-space form:
    every fit against the oracle, and two passes bit for bit equal."""
    import torch
    rng = np.random.default_rng(31)
    parts = []
    for k in range(700):
        m = 40 + (k * 53) % 160
        t = rng.uniform(0, 1, m)
        y = (1.0 + 0.5 * t) / (1.0 + 0.2 * t) * (1.0 + 0.005 * rng.normal(size=m))
        parts.append((np.stack([t, t]), y, 2, 4))
    batch = make_batch(parts)
    st = fit_and_compare(gpu_ctx, orc, batch, rp.RP_FP64, "unknown space, several per workgroup")
    assert np.all(st == rp.RP_FIT_RANK_DEFICIENT)
    db = rp.DeviceBatch(gpu_ctx, batch)
    c1, s1 = [t.clone() for t in db.fit()[:2]]
    c2, s2 = [t.clone() for t in db.fit()[:2]]
    torch.cuda.synchronize()
    assert torch.equal(c1, c2) and torch.equal(s1, s2)
