"""GPU parity of the fitting path against the FP64 CPU oracle.

Every call goes through the C ABI (ctypes binding).  Bars:
  * FP64 form: coefficient vector relative error (max-norm) <= 1e-9;
  * mixed forms: predictions f(u_i) at the samples relative error <= 1e-6
    (max over samples of |f_gpu - f_oracle| / max |f_oracle|), on fits whose
    fitted Q stays positive at every sample;
  * integer outputs (status) identical on unambiguous cases.
"""
import math
import sys

import numpy as np
import pytest

from paper_1906_00142_amd import rp
from paper_1906_00142_amd import workloads as W
from tests._parity import masked_pred_rel_err

pytestmark = pytest.mark.gpu

COEF_TOL = 1e-9
PRED_TOL = 1e-6


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def run_fit(ctx, batch, precision=rp.RP_FP64, max_refine=-1, tol=-1.0, gram_algo=rp.RP_GRAM_AUTO):
    import torch
    db = rp.DeviceBatch(ctx, batch)
    coef, status, resid, iters = db.fit(precision=precision, max_refine=max_refine, tol=tol,
                                        gram_algo=gram_algo)
    torch.cuda.synchronize()
    return (coef.cpu().numpy(), status.cpu().numpy(), resid.cpu().numpy(),
            iters.cpu().numpy(), db.plan.coef_off)


def coef_rel_err(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


def pred_rel_err(orc, batch, f, ca, cb):
    u, y = batch.fit_samples(f)
    v, d = int(batch.nvars[f]), int(batch.deg_num[f])
    pa = orc.eval_rational(v, d, d, ca, u)
    pb = orc.eval_rational(v, d, d, cb, u)
    return np.max(np.abs(pa - pb)) / np.max(np.abs(pb))


@pytest.mark.parametrize("algo", [rp.RP_GRAM_MOMENTS, rp.RP_GRAM_MFMA])
@pytest.mark.parametrize("v", [1, 2, 3, 4])
def test_fp64_parity_every_shape(gpu_ctx, orc, v, algo):
    # ragged sample counts: several chunks plus a partial tail for every tile size
    parts = [W.uniform_batch(3, m, v, d, 0.005, seed=100 * v + d)
             for d, m in ((1, 77), (2, 300), (3, 515), (4, 1100))]
    off = [0]
    xs, ys, nv, dg = [], [], [], []
    for b in parts:
        for f in range(b.num_fits):
            u, y = b.fit_samples(f)
            xs.append(u); ys.append(y); off.append(off[-1] + len(y))
            nv.append(v); dg.append(int(b.deg_num[f]))
    batch = W.FitBatch(len(nv), v, np.array(off, dtype=np.int64), np.array(nv, np.int32),
                       np.array(dg, np.int32), np.array(dg, np.int32),
                       np.concatenate(xs, axis=1), np.concatenate(ys), 0.005)
    say("fp64 parity v", v, "fits", batch.num_fits, "gram", algo)
    coef, status, resid, iters, coff = run_fit(gpu_ctx, batch, gram_algo=algo)
    ocoef, ocoff, ostatus, oresid = orc.fit_batch(batch, nthreads=8)
    np.testing.assert_array_equal(coff, ocoff)
    for f in range(batch.num_fits):
        a, b = coef[coff[f]:coff[f + 1]], ocoef[coff[f]:coff[f + 1]]
        assert coef_rel_err(a, b) <= COEF_TOL, (f, coef_rel_err(a, b))
        assert status[f] == ostatus[f], (f, status[f], ostatus[f])
        np.testing.assert_allclose(resid[f], oresid[f], rtol=1e-9)


def test_fp64_exact_recovery_of_planted(gpu_ctx, orc):
    from conftest import planted_in_order
    batch = W.uniform_batch(8, 700, 3, 3, 0.0, seed=5)
    coef, status, resid, iters, coff = run_fit(gpu_ctx, batch)
    for f in range(batch.num_fits):
        want = planted_in_order(orc, batch.planted[f])
        assert coef_rel_err(coef[coff[f]:coff[f + 1]], want) <= 1e-9
        assert status[f] == 0
        assert resid[f] <= 1e-10 * np.linalg.norm(batch.fit_samples(f)[1])


@pytest.mark.parametrize("precision", [rp.RP_MIXED_FP32, rp.RP_MIXED_BF16])
def test_mixed_precision_predictions(gpu_ctx, orc, precision):
    """Every fit is full rank (oracle status 0, or 4: Q <= 0 at a sample):
    predictions within 1e-6 over the samples where the oracle's |Q| >= 1e-3,
    coefficients within 1e-6, statuses equal."""
    batch = W.uniform_batch(24, 2048, 3, 3, 0.005, seed=77)
    coef, status, resid, iters, coff = run_fit(gpu_ctx, batch, precision=precision,
                                               max_refine=40, tol=1e-12)
    ocoef, ocoff, ostatus, oresid = orc.fit_batch(batch, nthreads=8)
    worst, checked = 0.0, 0
    for f in range(batch.num_fits):
        a, b = coef[coff[f]:coff[f + 1]], ocoef[coff[f]:coff[f + 1]]
        assert ostatus[f] in (0, 4) and status[f] == ostatus[f], (f, status[f], ostatus[f])
        u, _ = batch.fit_samples(f)
        e = masked_pred_rel_err(orc, u, 3, 3, 3, a, b)
        worst = max(worst, e)
        checked += 1
        assert e <= PRED_TOL, (f, e, iters[f])
        assert coef_rel_err(a, b) <= 1e-6, (f, coef_rel_err(a, b))
        np.testing.assert_allclose(resid[f], oresid[f], rtol=1e-6)
    say("precision", precision, "checked", checked, "worst pred err", worst,
        "statuses", np.bincount(ostatus, minlength=6).tolist(),
        "iters", np.percentile(iters, [50, 100]))


def test_edge_cases(gpu_ctx, orc):
    rng = np.random.default_rng(3)
    us, ys = [], []
    # 0: empty fit; 1: underdetermined (10 samples, 11 unknowns); 2: NaN sample;
    # 3: collinear variables (rank deficient); 4: exactly determined
    us.append(np.zeros((2, 0))); ys.append(np.zeros(0))
    u = rng.uniform(0, 1, (2, 10)); us.append(u); ys.append(1.0 + u[0] * u[1])
    u = rng.uniform(0, 1, (2, 50)); y = 1.0 + u[0]; y[7] = np.nan; us.append(u); ys.append(y)
    t = rng.uniform(0, 1, 60); us.append(np.stack([t, t])); ys.append(1.0 + 0.5 * t + 0.01 * rng.normal(size=60))
    pb = W.interpolation_batch(1, 2, 2, seed=9); u, y = pb.fit_samples(0); us.append(u); ys.append(y)
    off = np.zeros(len(us) + 1, dtype=np.int64)
    np.cumsum([len(y) for y in ys], out=off[1:])
    batch = W.FitBatch(len(us), 2, off, np.full(len(us), 2, np.int32), np.full(len(us), 2, np.int32),
                       np.full(len(us), 2, np.int32), np.concatenate(us, axis=1), np.concatenate(ys), 0.0)
    coef, status, resid, iters, coff = run_fit(gpu_ctx, batch)
    ocoef, ocoff, ostatus, oresid = orc.fit_batch(batch)
    assert status.tolist()[:4] == [2, 2, 3, 1] and ostatus.tolist()[:4] == [2, 2, 3, 1]
    assert np.all(coef[coff[0]:coff[1]] == 0.0)
    assert np.all(np.isnan(coef[coff[2]:coff[3]]))
    # rank deficient: the minimum-norm least-squares minimiser on both sides
    np.testing.assert_allclose(resid[3], oresid[3], rtol=1e-7)
    assert coef_rel_err(coef[coff[3]:coff[4]], ocoef[coff[3]:coff[4]]) <= COEF_TOL
    # square system: exact interpolation
    assert status[4] == 0 and resid[4] <= 1e-9 * np.linalg.norm(ys[4])
    assert coef_rel_err(coef[coff[4]:coff[5]], ocoef[coff[4]:coff[5]]) <= COEF_TOL
    # underdetermined: the minimum-norm interpolant
    assert resid[1] <= 1e-8 * np.linalg.norm(ys[1])
    assert coef_rel_err(coef[coff[1]:coff[2]], ocoef[coff[1]:coff[2]]) <= COEF_TOL


@pytest.mark.parametrize("vd", [(3, 4), (4, 3), (4, 4)])
@pytest.mark.parametrize("precision", [rp.RP_FP64, rp.RP_MIXED_FP32, rp.RP_MIXED_BF16])
def test_edge_cases_larger_models(gpu_ctx, orc, vd, precision):
    """Models of more than 39 unknowns (the workgroup sweep; FP64 through the
    separate sweep kernel): an empty fit, a NaN output sample, an infinite
    input, and a planted fit, side by side in one bucket."""
    v, d = vd
    nc = 2 * math.comb(v + d, d) - 1
    rng = np.random.default_rng(40 + 10 * v + d)
    us, ys = [], []
    us.append(np.zeros((v, 0))); ys.append(np.zeros(0))
    u = rng.uniform(0, 1, (v, nc + 50)); y = 1.0 + u.sum(axis=0); y[nc // 2] = np.nan; us.append(u); ys.append(y)
    u = rng.uniform(0, 1, (v, nc + 60)); u[v - 1, 3] = np.inf; us.append(u); ys.append(1.0 + u[0])
    pl = W.plant(rng, v, d, d)
    u = rng.uniform(0, 1, (v, 3 * nc)); us.append(u); ys.append(pl.value(u) * (1.0 + 0.005 * rng.normal(size=3 * nc)))
    off = np.zeros(len(us) + 1, dtype=np.int64)
    np.cumsum([len(y) for y in ys], out=off[1:])
    n = len(us)
    batch = W.FitBatch(n, v, off, np.full(n, v, np.int32), np.full(n, d, np.int32), np.full(n, d, np.int32),
                       np.concatenate(us, axis=1), np.concatenate(ys), 0.005)
    coef, status, resid, iters, coff = run_fit(gpu_ctx, batch, precision=precision)
    ocoef, ocoff, ostatus, oresid = orc.fit_batch(batch)
    say("larger-model edge cases", vd, precision, status.tolist(), ostatus.tolist())
    assert status.tolist()[:3] == [2, 3, 3] and ostatus.tolist()[:3] == [2, 3, 3]
    assert np.all(coef[coff[0]:coff[1]] == 0.0)
    assert np.all(np.isnan(coef[coff[1]:coff[2]])) and np.all(np.isnan(coef[coff[2]:coff[3]]))
    assert np.isnan(resid[1]) and np.isnan(resid[2])
    assert status[3] == ostatus[3]
    a, b = coef[coff[3]:coff[4]], ocoef[coff[3]:coff[4]]
    if precision == rp.RP_FP64:
        assert coef_rel_err(a, b) <= COEF_TOL
    else:
        assert pred_rel_err(orc, batch, 3, a, b) <= 1e-6


def test_empty_batch_and_uneven_mix(gpu_ctx, orc):
    import torch
    empty = W.FitBatch(0, 1, np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.int32),
                       np.zeros(0, np.int32), np.zeros((1, 1)), np.zeros(1), 0.0)
    db = rp.DeviceBatch(gpu_ctx, empty)
    assert db.plan.num_coefs == 0
    torch.cuda.synchronize()
    batch = W.uneven_batch(num_fits=40, m_lo=16, m_hi=1500, seed=31)
    coef, status, resid, iters, coff = run_fit(gpu_ctx, batch)
    ocoef, ocoff, ostatus, oresid = orc.fit_batch(batch, nthreads=8)
    m = np.diff(batch.sample_off)
    for f in range(batch.num_fits):
        a, b = coef[coff[f]:coff[f + 1]], ocoef[coff[f]:coff[f + 1]]
        # full rank, rank deficient and underdetermined alike: one minimiser
        assert coef_rel_err(a, b) <= COEF_TOL, (f, batch.nvars[f], batch.deg_num[f], m[f], status[f])
        assert status[f] == ostatus[f], (f, status[f], ostatus[f])
    say("uneven mix statuses", np.bincount(status, minlength=6).tolist())


def test_deterministic_and_order_independent(gpu_ctx):
    batch = W.uniform_batch(16, 900, 2, 3, 0.01, seed=8)
    c1, s1, r1, _, coff = run_fit(gpu_ctx, batch)
    c2, s2, r2, _, _ = run_fit(gpu_ctx, batch)
    np.testing.assert_array_equal(c1, c2)
    perm = np.random.default_rng(0).permutation(batch.num_fits)
    xs, ys, off = [], [], [0]
    for f in perm:
        u, y = batch.fit_samples(f); xs.append(u); ys.append(y); off.append(off[-1] + len(y))
    pb = W.FitBatch(batch.num_fits, 2, np.array(off, np.int64), batch.nvars[perm], batch.deg_num[perm],
                    batch.deg_den[perm], np.concatenate(xs, axis=1), np.concatenate(ys), 0.01)
    c3, s3, r3, _, coff3 = run_fit(gpu_ctx, pb)
    for k, f in enumerate(perm):
        np.testing.assert_array_equal(c3[coff3[k]:coff3[k + 1]], c1[coff[f]:coff[f + 1]])


@pytest.mark.parametrize("precision,dtype_name", [(rp.RP_FP64, "float64"), (rp.RP_MIXED_FP32, "float32"),
                                                  (rp.RP_MIXED_BF16, "bfloat16")])
def test_assemble_design(gpu_ctx, orc, precision, dtype_name):
    import torch
    batch = W.uneven_batch(num_fits=12, m_lo=8, m_hi=300, seed=12)
    db = rp.DeviceBatch(gpu_ctx, batch)
    dt = getattr(torch, dtype_name)
    A = torch.empty(int(db.plan.a_off[-1]), dtype=dt, device=db.device)
    rhs = torch.empty(batch.total_samples, dtype=dt, device=db.device)
    rp.rp_assemble_design(db.plan, db.x, db.ld_x, db.y, precision, A, rhs)
    torch.cuda.synchronize()
    An = A.to(torch.float64).cpu().numpy()
    rn = rhs.to(torch.float64).cpu().numpy()
    for f in range(batch.num_fits):
        u, y = batch.fit_samples(f)
        v, d = int(batch.nvars[f]), int(batch.deg_num[f])
        Ao, bo = orc.design(u, y, d, d)
        got = An[db.plan.a_off[f]:db.plan.a_off[f + 1]].reshape(Ao.shape)
        want = torch.from_numpy(Ao).to(dt).to(torch.float64).numpy()
        rel = {"float64": 4e-16 * 8, "float32": 2.0 ** -23, "bfloat16": 2.0 ** -7}[dtype_name]
        np.testing.assert_allclose(got, want, rtol=rel, atol=0)
        a, b = int(batch.sample_off[f]), int(batch.sample_off[f + 1])
        np.testing.assert_array_equal(rn[a:b], torch.from_numpy(bo).to(dt).to(torch.float64).numpy())


@pytest.mark.parametrize("precision,algo,rtol", [(rp.RP_FP64, rp.RP_GRAM_MOMENTS, 1e-13),
                                                 (rp.RP_FP64, rp.RP_GRAM_MFMA, 1e-13),
                                                 (rp.RP_MIXED_FP32, rp.RP_GRAM_AUTO, 2e-6),
                                                 (rp.RP_MIXED_BF16, rp.RP_GRAM_AUTO, 3e-2)])
def test_batched_gram_against_design(gpu_ctx, orc, precision, algo, rtol):
    """rp_gram: packed [A b]^T [A b] per fit vs the oracle's design (NumPy product)."""
    import torch
    batch = W.uneven_batch(num_fits=20, m_lo=16, m_hi=900, seed=17)
    db = rp.DeviceBatch(gpu_ctx, batch)
    gram = torch.full((int(db.plan.gram_off[-1]),), np.nan, dtype=torch.float64, device=db.device)
    rp.rp_gram(db.plan, db.x, db.ld_x, db.y, precision, gram, gram_algo=algo)
    torch.cuda.synchronize()
    g = gram.cpu().numpy()
    for f in range(batch.num_fits):
        u, y = batch.fit_samples(f)
        d = int(batch.deg_num[f])
        A, b = orc.design(u, y, d, d)
        Ab = np.concatenate([A, b[:, None]], axis=1)
        G = Ab.T @ Ab
        n = G.shape[0]
        got = np.zeros_like(G)
        seg = g[db.plan.gram_off[f]:db.plan.gram_off[f + 1]]
        assert len(seg) == n * (n + 1) // 2
        for i in range(n):
            got[i, :i + 1] = seg[i * (i + 1) // 2: i * (i + 1) // 2 + i + 1]
        low = np.tril_indices(n)
        scale = np.sqrt(np.outer(np.diag(G), np.diag(G)))[low]
        err = np.max(np.abs(got[low] - G[low]) / np.maximum(scale, 1e-300))
        assert err <= rtol, (f, err)


@pytest.mark.parametrize("algo", [rp.RP_GRAM_MOMENTS, rp.RP_GRAM_MFMA])
def test_jacobian_gram_against_definition(gpu_ctx, orc, algo):
    """rp_gram_jacobian: packed [J r]^T [J r] at given coefficients, with
    J = (1/Q)[m, -f m'] and r = y - f written out from the oracle's monomial
    design, on an uneven batch at the planted coefficients (Q >= 1)."""
    import torch
    from conftest import planted_in_order
    batch = W.uneven_batch(num_fits=20, m_lo=16, m_hi=900, seed=19)
    db = rp.DeviceBatch(gpu_ctx, batch)
    coff = db.plan.coef_off
    coef = np.concatenate([planted_in_order(orc, batch.planted[f]) for f in range(batch.num_fits)])
    assert len(coef) == coff[-1]
    c_dev = torch.from_numpy(coef).to(db.device)
    gram = torch.full((int(db.plan.gram_off[-1]),), np.nan, dtype=torch.float64, device=db.device)
    rp.rp_gram_jacobian(db.plan, db.x, db.ld_x, db.y, c_dev, gram, gram_algo=algo)
    torch.cuda.synchronize()
    g = gram.cpu().numpy()
    for f in range(batch.num_fits):
        u, y = batch.fit_samples(f)
        d = int(batch.deg_num[f])
        A, _ = orc.design(u, y, d, d)
        na = A.shape[1] // 2 + 1
        mo = A[:, :na]
        c = coef[coff[f]:coff[f + 1]]
        N = mo @ c[:na]
        Q = 1.0 + mo[:, 1:] @ c[na:]
        fv = N / Q
        J = np.concatenate([mo / Q[:, None], -(fv / Q)[:, None] * mo[:, 1:]], axis=1)
        Jr = np.concatenate([J, (y - fv)[:, None]], axis=1)
        G = Jr.T @ Jr
        n = G.shape[0]
        seg = g[db.plan.gram_off[f]:db.plan.gram_off[f + 1]]
        assert len(seg) == n * (n + 1) // 2
        got = np.zeros_like(G)
        for i in range(n):
            got[i, :i + 1] = seg[i * (i + 1) // 2: i * (i + 1) // 2 + i + 1]
        low = np.tril_indices(n)
        scale = np.sqrt(np.outer(np.diag(G), np.diag(G)))[low]
        err = np.max(np.abs(got[low] - G[low]) / np.maximum(scale, 1e-300))
        assert err <= 1e-12, (f, err)
        # the corner entry is the true loss
        np.testing.assert_allclose(got[-1, -1], np.sum((fv - y) ** 2), rtol=1e-12)


UNEQUAL = [(v, dn, dq) for v in (1, 2, 3) for dn, dq in ((1, 2), (2, 1), (2, 3), (3, 2))]


def test_unequal_degree_shapes_accepted_and_others_refused(gpu_ctx):
    for v, dn, dq in UNEQUAL + [(4, 4, 4)]:
        p = rp.Plan(gpu_ctx, np.array([0, 50], np.int64), [v], [dn], [dq])
        p.close()
    for v, dn, dq in ((4, 2, 3), (2, 1, 3), (1, 4, 3), (3, 3, 1)):
        with pytest.raises(rp.RpError) as ei:
            rp.Plan(gpu_ctx, np.array([0, 50], np.int64), [v], [dn], [dq])
        assert ei.value.code == rp.RP_EUNSUPPORTED


@pytest.mark.parametrize("v,dn,dq", UNEQUAL)
def test_unequal_degrees_every_form(gpu_ctx, orc, v, dn, dq):
    """Numerator and denominator of different degrees (the Section 4.2
    display bounds them separately): FP64 coefficients (moment and MFMA
    Grams) within 1e-9 of the oracle with equal statuses; mixed forms'
    predictions within 1e-6 where the oracle's |Q| >= 1e-3."""
    batch = W.uniform_batch(40, 600, v, dn, 0.005, seed=60 + 7 * v + dn, deg_den=dq)
    ocoef, ocoff, ost, ores = orc.fit_batch(batch, nthreads=8)
    for algo in (rp.RP_GRAM_MOMENTS, rp.RP_GRAM_MFMA):
        coef, status, resid, iters, coff = run_fit(gpu_ctx, batch, gram_algo=algo)
        assert np.array_equal(coff, ocoff)
        for f in range(batch.num_fits):
            a, b = coef[coff[f]:coff[f + 1]], ocoef[coff[f]:coff[f + 1]]
            assert status[f] == ost[f], (f, status[f], ost[f])
            assert coef_rel_err(a, b) <= COEF_TOL, (algo, f, coef_rel_err(a, b))
            np.testing.assert_allclose(resid[f], ores[f], rtol=1e-9)
    for prec in (rp.RP_MIXED_FP32, rp.RP_MIXED_BF16):
        coef, status, resid, iters, coff = run_fit(gpu_ctx, batch, precision=prec)
        for f in range(batch.num_fits):
            a, b = coef[coff[f]:coff[f + 1]], ocoef[coff[f]:coff[f + 1]]
            u, _ = batch.fit_samples(f)
            assert masked_pred_rel_err(orc, u, v, dn, dq, a, b) <= PRED_TOL, (prec, f)


def test_unequal_degrees_gram_loss_and_refinement(gpu_ctx, orc):
    """The moment Gram of an unequal-degree model against its materialised
    design, the FP32 loss against the oracle's, and the LM refinement."""
    import torch
    v, dn, dq = 2, 3, 2
    batch = W.uniform_batch(12, 500, v, dn, 0.005, seed=71, deg_den=dq)
    db = rp.DeviceBatch(gpu_ctx, batch)
    gram = torch.empty(int(db.plan.gram_off[-1]), dtype=torch.float64, device=db.device)
    rp.rp_gram(db.plan, db.x, db.ld_x, db.y, rp.RP_FP64, gram, gram_algo=rp.RP_GRAM_MOMENTS)
    coef, status, resid, iters = db.fit()
    torch.cuda.synchronize()
    g = gram.cpu().numpy()
    coff = db.plan.coef_off
    for f in range(batch.num_fits):
        u, y = batch.fit_samples(f)
        A, rhs = orc.design(u, y, dn, dq)
        Au = np.column_stack([A, rhs])
        G = Au.T @ Au
        nu = G.shape[0]
        packed = np.concatenate([G[i, :i + 1] for i in range(nu)])
        got = g[db.plan.gram_off[f]:db.plan.gram_off[f + 1]]
        np.testing.assert_allclose(got, packed, rtol=1e-12, atol=1e-12 * np.abs(packed).max())
    c = coef.cpu().numpy()
    start = coef.clone()
    st = torch.zeros(batch.num_fits, dtype=torch.int32, device=db.device)
    loss = torch.zeros(batch.num_fits, dtype=torch.float64, device=db.device)
    K = 60
    rp.rp_refine_rational(db.plan, db.x, db.ld_x, db.y, start, st, loss, max_iter=K)
    torch.cuda.synchronize()
    s, L = start.cpu().numpy(), loss.cpu().numpy()
    slow = 0
    for f in range(batch.num_fits):
        u, y = batch.fit_samples(f)
        c0 = c[coff[f]:coff[f + 1]]
        oc, oL, oit = orc.refine(u, y, dn, dq, c0, max_iter=K, rtol=1e-14)
        if oit < K:
            # converged: the same minimum
            np.testing.assert_allclose(L[f], oL, rtol=1e-9)
            assert np.max(np.abs(s[coff[f]:coff[f + 1]] - oc)) <= 1e-6 * np.max(np.abs(oc))
            continue
        # still descending a flat valley after K steps: rounding moves the
        # accept/reject decisions, so the GPU must lie on the oracle's path
        # within ten steps either way
        slow += 1
        _, lo, _ = orc.refine(u, y, dn, dq, c0, max_iter=K + 10, rtol=1e-14)
        _, hi, _ = orc.refine(u, y, dn, dq, c0, max_iter=K - 10, rtol=1e-14)
        assert lo * (1 - 1e-9) <= L[f] <= hi * (1 + 1e-9), (f, L[f], lo, oL, hi)
    assert slow < batch.num_fits
