"""GPU parity of rational-program evaluation and argmin against the oracle.

Selection bar: the GPU's index equals the oracle's, unless the oracle's two
best values are within 1e-6 relative; then any candidate whose oracle value is
within 1e-6 of the oracle's best is accepted.  Values: FP64 form within
1e-12 relative of the oracle (the two differ only in rounding order).
"""
import sys

import numpy as np
import pytest

from conftest import planted_in_order
from paper_1906_00142_amd import rp
from paper_1906_00142_amd import workloads as W

pytestmark = pytest.mark.gpu
TIE = 1e-6


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def program_arrays(orc, metrics):
    deg = np.array([m.deg_num for m in metrics], dtype=np.int32)
    coefs = [planted_in_order(orc, m) for m in metrics]
    off = np.zeros(len(coefs) + 1, dtype=np.int64)
    np.cumsum([len(c) for c in coefs], out=off[1:])
    return deg, np.concatenate(coefs), off


def gpu_argmin(ctx, template, nvars, deg, coef, off, scale, n_grid, cand, hw=None, P=1,
               precision=rp.RP_FP64, want_values=False):
    import torch
    dev = torch.device("cuda", 0)
    coef_t = torch.from_numpy(coef).to(dev)
    hw_t = None if hw is None else torch.from_numpy(np.ascontiguousarray(hw, dtype=np.float64)).to(dev)
    prog = rp.Program(ctx, template, nvars, deg, deg, off, coef_t, scale, hw_t, num_programs=P)
    n_t = torch.from_numpy(np.asarray(n_grid, dtype=np.float64)).to(dev)
    c_t = torch.from_numpy(np.ascontiguousarray(cand, dtype=np.int32)).to(dev)
    num_n = len(n_grid)
    am = torch.full((P, num_n), -7, dtype=torch.int32, device=dev)
    best = torch.zeros((P, num_n), dtype=torch.float64, device=dev)
    second = torch.zeros((P, num_n), dtype=torch.float64, device=dev)
    values = (torch.zeros((P, num_n, len(cand)), dtype=torch.float64, device=dev)
              if want_values else None)
    rp.rp_eval_program_argmin(prog, n_t, c_t, am, best, second, values, precision=precision)
    torch.cuda.synchronize()
    out = (am.cpu().numpy(), best.cpu().numpy(), second.cpu().numpy())
    if want_values:
        out = out + (values.cpu().numpy(),)
    return out


def check_selection(orc_prog, p, n_grid, cand, am, best, oam, obest, osecond, vtol=1e-12):
    for j, n in enumerate(n_grid):
        if oam[p, j] < 0:
            assert am[p, j] == -1
            continue
        if am[p, j] != oam[p, j]:
            assert osecond[p, j] <= obest[p, j] * (1 + TIE), (j, am[p, j], oam[p, j])
            v = orc_prog.value(p, n, cand[am[p, j]])
            assert v <= obest[p, j] * (1 + TIE)
        np.testing.assert_allclose(best[p, j], orc_prog.value(p, n, cand[am[p, j]]), rtol=vtol)


def test_single_template_tiny_workload(gpu_ctx, orc):
    b = W.tiny_fit()
    deg, coef, off = program_arrays(orc, b.planted)
    scale = [2.0 ** 14, 1024.0]
    n_grid = W.tiny_grid(64)
    cand = (32 * np.arange(1, 33)).astype(np.int32).reshape(-1, 1)
    am, best, second, values = gpu_argmin(gpu_ctx, rp.RP_TEMPLATE_SINGLE, 2, deg, coef, off, scale,
                                          n_grid, cand, want_values=True)
    prog = orc.Program(orc.TEMPLATE_SINGLE, 2, deg, deg, coef, off, scale=scale)
    oam, obest, osecond = orc.argmin(prog, n_grid, cand)
    check_selection(prog, 0, n_grid, cand, am, best, oam, obest, osecond)
    np.testing.assert_allclose(second, osecond, rtol=1e-12)
    for j in (0, 17, 63):
        ov = [prog.value(0, n_grid[j], c) for c in cand]
        np.testing.assert_allclose(values[0, j], ov, rtol=1e-12)


def test_mwpcwp_program_full_grid(gpu_ctx, orc):
    pw = W.program_workload()
    deg, coef, off = program_arrays(orc, pw.metrics)
    cand = rp.rp_candidates_2d(1024, 64)
    assert len(cand) == 230
    am, best, second = gpu_argmin(gpu_ctx, rp.RP_TEMPLATE_MWPCWP, 3, deg, coef, off, pw.scales,
                                  pw.n_grid, cand, hw=pw.hw)
    prog = orc.Program(orc.TEMPLATE_MWPCWP, 3, deg, deg, coef, off, hw=pw.hw, hw_stride=17,
                       scale=pw.scales)
    pick = np.linspace(0, len(pw.n_grid) - 1, 96).astype(int)
    oam, obest, osecond = orc.argmin(prog, pw.n_grid[pick], cand)
    check_selection(prog, 0, pw.n_grid[pick], cand, am[:, pick], best[:, pick], oam, obest, osecond)
    chosen = {tuple(cand[k]) for k in am[0]}
    say("distinct selections over 1024 n:", len(chosen))
    assert len(chosen) >= 2


def test_mwpcwp_fp32_scan_rescored(gpu_ctx, orc):
    pw = W.program_workload()
    deg, coef, off = program_arrays(orc, pw.metrics)
    cand = rp.rp_candidates_2d(1024, 64)
    am, best, second = gpu_argmin(gpu_ctx, rp.RP_TEMPLATE_MWPCWP, 3, deg, coef, off, pw.scales,
                                  pw.n_grid, cand, hw=pw.hw, precision=rp.RP_MIXED_FP32)
    prog = orc.Program(orc.TEMPLATE_MWPCWP, 3, deg, deg, coef, off, hw=pw.hw, hw_stride=17,
                       scale=pw.scales)
    pick = np.linspace(0, len(pw.n_grid) - 1, 96).astype(int)
    oam, obest, osecond = orc.argmin(prog, pw.n_grid[pick], cand)
    check_selection(prog, 0, pw.n_grid[pick], cand, am[:, pick], best[:, pick], oam, obest, osecond)


def test_ties_invalid_and_empty(gpu_ctx, orc):
    cand = (32 * np.arange(1, 33)).astype(np.int32).reshape(-1, 1)
    const = np.array([1.0, 0.0, 0.0, 0.0, 0.0])
    deg = np.array([1], np.int32)
    off = np.array([0, 5], np.int64)
    am, best, second = gpu_argmin(gpu_ctx, rp.RP_TEMPLATE_SINGLE, 2, deg, const, off, [1.0, 1024.0],
                                  [1.0, 2.0, 3.0], cand)
    assert am.tolist() == [[0, 0, 0]] and np.all(best == 1.0) and np.all(second == 1.0)
    bad = np.array([1.0, 0.0, 0.0, 0.0, -2.0])          # Q = 1 - 2 u_b <= 0 for b >= 512
    am, best, second = gpu_argmin(gpu_ctx, rp.RP_TEMPLATE_SINGLE, 2, deg, bad, off, [1.0, 1024.0],
                                  [1.0], cand[15:])
    assert am.tolist() == [[-1]] and np.isinf(best[0, 0]) and np.isinf(second[0, 0])
    am, best, second = gpu_argmin(gpu_ctx, rp.RP_TEMPLATE_SINGLE, 2, deg, const, off, [1.0, 1024.0],
                                  [1.0, 5.0], cand[:0])
    assert am.tolist() == [[-1, -1]]


def test_many_single_programs(gpu_ctx, orc):
    """Many fitted programs over a 2-D candidate grid at four data sizes."""
    batch = W.uniform_batch(40, 200, 3, 2, 0.0, seed=4)
    coefs = [planted_in_order(orc, p) for p in batch.planted]
    coef = np.concatenate(coefs)
    off = np.zeros(41, np.int64)
    np.cumsum([len(c) for c in coefs], out=off[1:])
    deg = np.full(40, 2, np.int32)
    g = np.arange(1, 65)
    cand = np.stack(np.meshgrid(g, g, indexing="ij"), axis=-1).reshape(-1, 2).astype(np.int32)
    scale = [4096.0, 64.0, 64.0]
    n_grid = np.array([1024.0, 2048.0, 3072.0, 4096.0])
    am, best, second = gpu_argmin(gpu_ctx, rp.RP_TEMPLATE_SINGLE, 3, deg, coef, off, scale, n_grid,
                                  cand, P=40)
    prog = orc.Program(orc.TEMPLATE_SINGLE, 3, deg, deg, coef, off, scale=scale, num_programs=40)
    oam, obest, osecond = orc.argmin(prog, n_grid, cand)
    for p in range(40):
        check_selection(prog, p, n_grid, cand, am, best, oam, obest, osecond)


# --------------------------------------------------------------------------
# occupancy program and selection with a second metric (Section 2 Example 1,
# equation (occupancy); Section 3.3 step 5)
# --------------------------------------------------------------------------

def _dev_program(ctx, template, nvars, deg, den, coef, off, scale, hw=None, P=1):
    import torch
    dev = torch.device("cuda", 0)
    coef_t = torch.from_numpy(np.ascontiguousarray(coef, dtype=np.float64)).to(dev)
    hw_t = None if hw is None else torch.from_numpy(np.ascontiguousarray(hw, dtype=np.float64)).to(dev)
    return rp.Program(ctx, template, nvars, deg, den, off, coef_t, scale, hw_t, num_programs=P)


def gpu_select(prog, n_grid, cand, sense, tie=None, tie_sense=rp.RP_SELECT_MAX,
               precision=rp.RP_FP64):
    import torch
    dev = torch.device("cuda", 0)
    n_t = torch.from_numpy(np.asarray(n_grid, dtype=np.float64)).to(dev)
    c_t = torch.from_numpy(np.ascontiguousarray(cand, dtype=np.int32)).to(dev)
    P, num_n = prog.num_programs, len(n_grid)
    ch = torch.full((P, num_n), -7, dtype=torch.int32, device=dev)
    best = torch.zeros((P, num_n), dtype=torch.float64, device=dev)
    second = torch.zeros((P, num_n), dtype=torch.float64, device=dev)
    rp.rp_eval_program_select(prog, n_t, c_t, ch, best, second, sense=sense, tie_prog=tie,
                              tie_sense=tie_sense, precision=precision)
    torch.cuda.synchronize()
    return ch.cpu().numpy(), best.cpu().numpy(), second.cpu().numpy()


def _occ_arrays(orc, ow):
    deg = np.array([m.deg_num for m in ow.metrics], np.int32)
    den = np.array([m.deg_den for m in ow.metrics], np.int32)
    coefs = [planted_in_order(orc, m) for m in ow.metrics]
    off = np.zeros(3, np.int64)
    np.cumsum([len(c) for c in coefs], out=off[1:])
    return deg, den, np.concatenate(coefs), off


@pytest.mark.parametrize("precision", [rp.RP_FP64, rp.RP_MIXED_FP32])
def test_occupancy_program_maximised(gpu_ctx, orc, precision):
    """The occupancy program of the MWP-CWP workload (its registers and LDS
    metrics), maximised over the 230 block formats at 96 data sizes."""
    ow = W.occupancy_workload()
    deg, den, coef, off = _occ_arrays(orc, ow)
    cand = rp.rp_candidates_2d(1024, 64)
    pick = np.linspace(0, len(ow.n_grid) - 1, 96).astype(int)
    n_grid = ow.n_grid[pick]
    prog = _dev_program(gpu_ctx, rp.RP_TEMPLATE_OCCUPANCY, 3, deg, den, coef, off, ow.scales, ow.hw)
    ch, best, second = gpu_select(prog, n_grid, cand, rp.RP_SELECT_MAX, precision=precision)
    oprog = orc.Program(orc.TEMPLATE_OCCUPANCY, 3, deg, den, coef, off, hw=ow.hw, hw_stride=17,
                        scale=ow.scales)
    och, obest, osecond = orc.select(oprog, n_grid, cand, sense=-1)
    # occupancy values are ratios of small integers: exact on both sides
    np.testing.assert_array_equal(best, obest)
    if precision == rp.RP_FP64:
        np.testing.assert_array_equal(ch, och)
        np.testing.assert_array_equal(second, osecond)
    else:
        # the FP32 scan keeps four candidates per data size; the one it picks is optimal
        for j, n in enumerate(n_grid):
            assert oprog.value(0, n, cand[ch[0, j]]) == obest[0, j], j
    ties = int(np.sum(osecond == obest))
    say("occupancy: distinct optima", len({tuple(cand[k]) for k in och[0]}), "tied data sizes", ties,
        "best range", obest.min(), obest.max())


def _product_and_occupancy(orc, P=2):
    """Primary: E = bx * by (every format with the same thread count ties);
    tie program: occupancy with registers 20 + 40 u_n + 4 bx + 3 by and LDS
    2048 + 4 bx by bytes (program 0), or registers 8 + 8 u_n + 0.05 bx +
    0.02 by and LDS 30000 + 60 by bytes (program 1)."""
    E2 = orc.monomials(3, 2)
    prim = np.array([1.0 if tuple(int(t) for t in e) == (0, 1, 1) else 0.0 for e in E2])
    E1 = orc.monomials(3, 1)
    regs = [dict(zip([(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)], r)) for r in
            ([20.0, 40.0, 4.0, 3.0], [8.0, 8.0, 0.05, 0.02])]
    lds = [{(0, 0, 0): 2048.0, (0, 1, 1): 4.0}, {(0, 0, 0): 30000.0, (0, 0, 1): 60.0}]
    tcoef, toff = [], [0]
    for p in range(P):
        r = np.array([regs[p].get(tuple(int(t) for t in e), 0.0) for e in E1])
        z = np.array([lds[p].get(tuple(int(t) for t in e), 0.0) for e in E2])
        tcoef += [r, z]
        toff += [toff[-1] + len(r), toff[-1] + len(r) + len(z)]
    pdeg = np.full(P, 2, np.int32)
    tdeg = np.array([1, 2] * P, np.int32)
    return (pdeg, np.zeros(P, np.int32), np.tile(prim, P), np.arange(P + 1, dtype=np.int64) * len(prim),
            tdeg, np.zeros(2 * P, np.int32), np.concatenate(tcoef), np.array(toff, np.int64))


@pytest.mark.parametrize("sense,tie_sense", [(1, -1), (1, 1), (-1, -1)])
def test_select_tie_break_by_occupancy(gpu_ctx, orc, sense, tie_sense):
    pdeg, pden, pcoef, poff, tdeg, tden, tcoef, toff = _product_and_occupancy(orc)
    scale = [2.0 ** 24, 1.0, 1.0]
    hw = np.tile(W.program_workload().hw, 2)
    cand = rp.rp_candidates_2d(1024, 64)
    n_grid = np.array([1024.0, 65536.0, 2.0 ** 20, 2.0 ** 24])
    prim = _dev_program(gpu_ctx, rp.RP_TEMPLATE_SINGLE, 3, pdeg, pden, pcoef, poff, scale, P=2)
    tie = _dev_program(gpu_ctx, rp.RP_TEMPLATE_OCCUPANCY, 3, tdeg, tden, tcoef, toff, scale, hw, P=2)
    ch, best, second = gpu_select(prim, n_grid, cand, sense, tie, tie_sense)
    oprim = orc.Program(orc.TEMPLATE_SINGLE, 3, pdeg, pden, pcoef, poff, scale=scale, num_programs=2)
    otie = orc.Program(orc.TEMPLATE_OCCUPANCY, 3, tdeg, tden, tcoef, toff, hw=hw, hw_stride=17,
                       scale=scale, num_programs=2)
    och, obest, osecond = orc.select(oprim, n_grid, cand, sense=sense, tie=otie, tie_sense=tie_sense)
    np.testing.assert_array_equal(ch, och)
    np.testing.assert_array_equal(best, obest)
    np.testing.assert_array_equal(second, osecond)
    # the tie program decided: without it the lowest index among the tied formats wins
    plain, _, _ = gpu_select(prim, n_grid, cand, sense)
    say("tie break", sense, tie_sense, "choices", [tuple(cand[k]) for k in ch[0]],
        "without", [tuple(cand[k]) for k in plain[0]])
    assert np.any(plain != ch)


def test_select_mwpcwp_with_occupancy_tie_program(gpu_ctx, orc):
    pw = W.program_workload()
    ow = W.occupancy_workload(pw)
    deg, coef, off = program_arrays(orc, pw.metrics)
    tdeg, tden, tcoef, toff = _occ_arrays(orc, ow)
    cand = rp.rp_candidates_2d(1024, 64)
    pick = np.linspace(0, len(pw.n_grid) - 1, 48).astype(int)
    n_grid = pw.n_grid[pick]
    prim = _dev_program(gpu_ctx, rp.RP_TEMPLATE_MWPCWP, 3, deg, deg, coef, off, pw.scales, pw.hw)
    tie = _dev_program(gpu_ctx, rp.RP_TEMPLATE_OCCUPANCY, 3, tdeg, tden, tcoef, toff, ow.scales, ow.hw)
    ch, best, second = gpu_select(prim, n_grid, cand, rp.RP_SELECT_MIN, tie, rp.RP_SELECT_MAX)
    oprim = orc.Program(orc.TEMPLATE_MWPCWP, 3, deg, deg, coef, off, hw=pw.hw, hw_stride=17,
                        scale=pw.scales)
    otie = orc.Program(orc.TEMPLATE_OCCUPANCY, 3, tdeg, tden, tcoef, toff, hw=ow.hw, hw_stride=17,
                       scale=ow.scales)
    och, obest, osecond = orc.select(oprim, n_grid, cand, sense=1, tie=otie, tie_sense=-1)
    check_selection(oprim, 0, n_grid, cand, ch, best, och, obest, osecond)
    # without exact ties of E the tie program changes nothing
    am, _, _ = gpu_argmin(gpu_ctx, rp.RP_TEMPLATE_MWPCWP, 3, deg, coef, off, pw.scales, n_grid, cand,
                          hw=pw.hw)
    tied = osecond[0] == obest[0]
    np.testing.assert_array_equal(ch[0][~tied], am[0][~tied])


def test_select_argument_checks(gpu_ctx, orc):
    pdeg, pden, pcoef, poff, tdeg, tden, tcoef, toff = _product_and_occupancy(orc, P=1)
    scale = [2.0 ** 24, 1.0, 1.0]
    hw = W.program_workload().hw
    cand = rp.rp_candidates_2d(1024, 64)
    prim = _dev_program(gpu_ctx, rp.RP_TEMPLATE_SINGLE, 3, pdeg, pden, pcoef, poff, scale)
    tie = _dev_program(gpu_ctx, rp.RP_TEMPLATE_OCCUPANCY, 3, tdeg, tden, tcoef, toff, scale, hw)
    with pytest.raises(rp.RpError, match="FP64"):
        gpu_select(prim, [1.0], cand, rp.RP_SELECT_MIN, tie, precision=rp.RP_MIXED_FP32)
    with pytest.raises(rp.RpError, match="sense"):
        gpu_select(prim, [1.0], cand, 0)
    pdeg2, pden2, pcoef2, poff2, _, _, _, _ = _product_and_occupancy(orc, P=2)
    prim2 = _dev_program(gpu_ctx, rp.RP_TEMPLATE_SINGLE, 3, pdeg2, pden2, pcoef2, poff2, scale, P=2)
    with pytest.raises(rp.RpError, match="num_programs"):
        gpu_select(prim2, [1.0], cand, rp.RP_SELECT_MIN, tie)
    with pytest.raises(rp.RpError, match="2 metrics"):
        _dev_program(gpu_ctx, rp.RP_TEMPLATE_OCCUPANCY, 3, pdeg, pden, pcoef, poff, scale, hw)
