"""The fit entry point that allocates nothing (rp_fit_uniform_static) against
rp_fit_rational on a plan of the same uniform batch: two calls in a row, the
second with a smaller batch, in a fresh process or after the other tests."""
import sys

import numpy as np
import pytest

from paper_1906_00142_amd import rp
from paper_1906_00142_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def run_both(ctx, batch, nvars, degree):
    import torch
    m = int(batch.sample_off[1])
    db = rp.DeviceBatch(ctx, batch)
    ref = db.fit()
    out = db.alloc_fit_outputs()
    for t in out:
        t.fill_(-7)
    say("static fit", batch.num_fits, "fits x", m, "samples, shape", nvars, degree)
    rp.rp_fit_uniform_static(ctx, batch.num_fits, m, nvars, degree, db.x, db.ld_x, db.y, *out)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in ref], [t.cpu().numpy() for t in out], db


@pytest.mark.parametrize("nvars,degree,fits,small", [(3, 3, 600, 97), (4, 4, 60, 9), (2, 1, 300, 5)])
def test_static_fit_equals_plan_fit(gpu_ctx, nvars, degree, fits, small):
    for k, F in enumerate((fits, small)):
        # the second call: fewer fits and other samples (a different seed)
        b = W.uniform_batch(F, 700 if k == 0 else 333, nvars, degree, 0.005, seed=31 + k)
        ref, got, db = run_both(gpu_ctx, b, nvars, degree)
        for name, r, g in zip(("coef", "status", "resid", "iters"), ref, got):
            assert np.array_equal(r, g), (name, F, np.flatnonzero(r != g)[:5])
        say("equal to the plan fit:", F, "fits, statuses", np.bincount(got[1], minlength=6).tolist())


def test_static_fit_flagged_fits_and_limits(gpu_ctx):
    """Underdetermined fits go through the re-solve list in the scratch too;
    a batch beyond the scratch is refused before anything runs."""
    import torch
    b = W.uniform_batch(40, 30, 3, 3, 0.005, seed=5)      # 30 samples < 39 unknowns
    ref, got, db = run_both(gpu_ctx, b, 3, 3)
    assert np.all(got[1] == rp.RP_FIT_UNDERDETERMINED)
    for name, r, g in zip(("coef", "status", "resid", "iters"), ref, got):
        assert np.array_equal(r, g), name
    x = torch.zeros((3, 6000 * 10), dtype=torch.float64, device=db.device)
    y = torch.zeros(6000 * 10, dtype=torch.float64, device=db.device)
    coef = torch.zeros(6000 * 39, dtype=torch.float64, device=db.device)
    st = torch.zeros(6000, dtype=torch.int32, device=db.device)
    rs = torch.zeros(6000, dtype=torch.float64, device=db.device)
    with pytest.raises(rp.RpError) as ei:
        rp.rp_fit_uniform_static(gpu_ctx, 6000, 10, 3, 3, x, 60000, y, coef, st, rs)
    assert "scratch" in str(ei.value)
