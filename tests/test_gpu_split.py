"""Decision nodes fitted from the samples (Section 3.2, third consequence) on
the GPU against the oracle's exhaustive search.

Bars: the split k equals the oracle's, except where the oracle's objective at
the GPU's split lies within 1e-9 relative of its minimum (two candidates
that FP64 rounding cannot order -- counted and printed); with k equal,
theta is bit-exact (the same two sorted inputs, the same formula), the
objective within 1e-9 relative, both sides' coefficients within 1e-9
relative (max norm) and the statuses equal."""
import sys

import numpy as np
import pytest

from paper_1906_00142_amd import rp
from paper_1906_00142_amd import workloads as W

pytestmark = pytest.mark.gpu

WIN = 1e-9


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def run_split(ctx, batch, nvars, degree, split_var, n_min):
    import torch
    dev = torch.device("cuda", ctx.device)
    x = torch.from_numpy(np.ascontiguousarray(batch.x)).to(dev)
    y = torch.from_numpy(np.ascontiguousarray(batch.y)).to(dev)
    m = int(batch.sample_off[1]) if batch.num_fits else 0
    sp = rp.Split(ctx, batch.num_fits, m, nvars, degree, split_var, n_min)
    out = sp.fit(x, int(batch.x.shape[1]), y)
    torch.cuda.synchronize()
    sp.close()
    return [t.cpu().numpy() for t in out]


def compare(orc, batch, got, degree, split_var, n_min):
    k, theta, cl, cr, sl, sr, obj = got
    nc = orc.num_coefs(int(batch.nvars[0]), degree, degree)
    same = near = 0
    worst = 0.0
    for f in range(batch.num_fits):
        u, y = batch.fit_samples(f)
        r = orc.split_fit(u, y, degree, split_var, n_min, want_all=True)
        # objectives at the rounding floor of the sums of squares are equal
        floor = 1e-24 * float(y @ y)
        if k[f] != r["k"]:
            assert r["k"] >= 0 and k[f] >= 0, (f, k[f], r["k"])
            assert r["obj_all"][k[f]] <= r["obj"] * (1 + WIN) + floor, (f, k[f], r["k"])
            near += 1
            continue
        same += 1
        assert sl[f] == r["status_l"] and sr[f] == r["status_r"], f
        if r["k"] < 0:
            assert np.isnan(theta[f]) and obj[f] == np.inf
            continue
        assert theta[f] == r["theta"], f
        np.testing.assert_allclose(obj[f], r["obj"], rtol=WIN, atol=floor)
        for a, o in ((cl[f * nc:(f + 1) * nc], r["coef_l"]), (cr[f * nc:(f + 1) * nc], r["coef_r"])):
            e = np.max(np.abs(a - o)) / np.max(np.abs(o))
            worst = max(worst, e)
            assert e <= 1e-9, (f, e)
    return same, near, worst


@pytest.mark.parametrize("nvars,degree,split_var", [(2, 2, 0), (2, 2, 1), (1, 3, 0), (3, 1, 2)])
def test_split_fit_against_oracle(gpu_ctx, orc, nvars, degree, split_var):
    sb = W.split_batch(48, 256, nvars, degree, split_var=split_var, sigma=0.005, seed=40 + split_var)
    n_min = orc.num_coefs(nvars, degree, degree)
    got = run_split(gpu_ctx, sb.batch, nvars, degree, split_var, n_min)
    same, near, worst = compare(orc, sb.batch, got, degree, split_var, n_min)
    # how often the least-squares split lands near the planted threshold
    # (information: with noise and similar pieces the best split may lie
    # elsewhere; parity with the oracle is what is checked)
    close = np.mean(np.abs(got[1] - sb.theta) < 0.05)
    say(f"split v={nvars} d={degree} s={split_var}: same split {same}, within the window {near}, "
        f"worst coefficient error {worst:.2e}, theta within 0.05 of planted on {close:.0%}")


def test_split_recovers_planted_nodes(gpu_ctx, orc):
    sb = W.split_batch(32, 300, 2, 2, split_var=1, sigma=0.0, gap=0.02, seed=44)
    got = run_split(gpu_ctx, sb.batch, 2, 2, 1, 11)
    k, theta = got[0], got[1]
    for f in range(sb.batch.num_fits):
        u, _ = sb.batch.fit_samples(f)
        assert k[f] == int((u[1] <= sb.theta[f]).sum())
        assert abs(theta[f] - sb.theta[f]) <= 0.03
    same, near, worst = compare(orc, sb.batch, got, 2, 1, 11)
    assert near == 0


def test_split_edge_cases(gpu_ctx, orc):
    """A node with a NaN sample, a node with many equal split values, and a
    minimum side size that leaves no candidate."""
    sb = W.split_batch(4, 120, 2, 1, split_var=0, sigma=0.01, seed=45)
    b = sb.batch
    b.y[b.sample_off[1] + 17] = np.nan
    a2 = int(b.sample_off[2])
    b.x[0, a2:a2 + 120] = np.round(b.x[0, a2:a2 + 120] * 6) / 6
    got = run_split(gpu_ctx, b, 2, 1, 0, 5)
    assert got[0][1] == -1 and got[4][1] == rp.RP_FIT_NONFINITE_INPUT
    compare(orc, b, got, 1, 0, 5)
    got = run_split(gpu_ctx, b, 2, 1, 0, 61)
    assert np.all(got[0] == -1) and np.all(np.isinf(got[6]))
    compare(orc, b, got, 1, 0, 61)
