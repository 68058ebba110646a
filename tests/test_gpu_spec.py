"""Specialised evaluators (code generation, Section 3.3 step 3; Section 4.3):
the run-time compiled evaluator against the table-driven one and the oracle.

Bars: values within 1e-14 relative of the table-driven evaluator (the same
arithmetic in the same order; only the compiler's contraction choices may
differ) and selections equal to the table-driven ones except where its best
two values are within 1e-12; selections checked against the oracle as in the
table-driven tests.
"""
import sys

import numpy as np
import pytest

from conftest import planted_in_order
from paper_1906_00142_amd import rp
from paper_1906_00142_amd import workloads as W
from test_gpu_eval import check_selection, program_arrays, _dev_program, _occ_arrays, gpu_select

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def spec_select(spec, P, n_grid, cand, sense):
    import torch
    dev = torch.device("cuda", 0)
    n_t = torch.from_numpy(np.asarray(n_grid, dtype=np.float64)).to(dev)
    c_t = torch.from_numpy(np.ascontiguousarray(cand, dtype=np.int32)).to(dev)
    num_n = len(n_grid)
    ch = torch.full((P, num_n), -7, dtype=torch.int32, device=dev)
    best = torch.zeros((P, num_n), dtype=torch.float64, device=dev)
    second = torch.zeros((P, num_n), dtype=torch.float64, device=dev)
    values = torch.zeros((P, num_n, len(cand)), dtype=torch.float64, device=dev)
    rp.rp_eval_spec_select(spec, n_t, c_t, ch, best, second, sense=sense, values=values)
    torch.cuda.synchronize()
    return ch.cpu().numpy(), best.cpu().numpy(), second.cpu().numpy(), values.cpu().numpy()


def table_select(prog, n_grid, cand, sense):
    import torch
    dev = torch.device("cuda", 0)
    n_t = torch.from_numpy(np.asarray(n_grid, dtype=np.float64)).to(dev)
    c_t = torch.from_numpy(np.ascontiguousarray(cand, dtype=np.int32)).to(dev)
    P, num_n = prog.num_programs, len(n_grid)
    ch = torch.full((P, num_n), -7, dtype=torch.int32, device=dev)
    best = torch.zeros((P, num_n), dtype=torch.float64, device=dev)
    second = torch.zeros((P, num_n), dtype=torch.float64, device=dev)
    values = torch.zeros((P, num_n, len(cand)), dtype=torch.float64, device=dev)
    rp.rp_eval_program_select(prog, n_t, c_t, ch, best, second, sense=sense, values=values)
    torch.cuda.synchronize()
    return ch.cpu().numpy(), best.cpu().numpy(), second.cpu().numpy(), values.cpu().numpy()


def compare(spec_out, table_out, label):
    sch, sb, ss, sv = spec_out
    tch, tb, ts, tv = table_out
    fin = np.isfinite(tv)
    np.testing.assert_array_equal(np.isfinite(sv), fin)
    rel = np.abs(sv[fin] - tv[fin]) / np.maximum(np.abs(tv[fin]), 1e-300)
    exact = float(np.mean(sv[fin] == tv[fin])) if fin.any() else 1.0
    say(label, "values", int(fin.sum()), "max rel diff", float(rel.max()) if rel.size else 0.0,
        "bit-equal fraction", exact)
    assert rel.size == 0 or rel.max() <= 1e-14
    clear = np.abs(ts - tb) > 1e-12 * np.abs(tb)
    np.testing.assert_array_equal(sch[clear], tch[clear])


def test_specialised_mwpcwp_program(gpu_ctx, orc):
    pw = W.program_workload()
    deg, coef, off = program_arrays(orc, pw.metrics)
    cand = rp.rp_candidates_2d(1024, 64)
    pick = np.linspace(0, len(pw.n_grid) - 1, 128).astype(int)
    n_grid = pw.n_grid[pick]
    prog = _dev_program(gpu_ctx, rp.RP_TEMPLATE_MWPCWP, 3, deg, deg, coef, off, pw.scales, pw.hw)
    spec = rp.Spec(prog)
    assert "rp_spec_eval" in spec.source() and "mwpcwp_cycles" in spec.source()
    s_out = spec_select(spec, 1, n_grid, cand, rp.RP_SELECT_MIN)
    t_out = table_select(prog, n_grid, cand, rp.RP_SELECT_MIN)
    compare(s_out, t_out, "mwpcwp")
    oprog = orc.Program(orc.TEMPLATE_MWPCWP, 3, deg, deg, coef, off, hw=pw.hw, hw_stride=17,
                        scale=pw.scales)
    sub = np.arange(0, 128, 4)
    och, obest, osecond = orc.argmin(oprog, n_grid[sub], cand)
    check_selection(oprog, 0, n_grid[sub], cand, s_out[0][:, sub], s_out[1][:, sub], och, obest, osecond)


def test_specialised_occupancy_program_maximised(gpu_ctx, orc):
    ow = W.occupancy_workload()
    deg, den, coef, off = _occ_arrays(orc, ow)
    cand = rp.rp_candidates_2d(1024, 64)
    n_grid = ow.n_grid[::16]
    prog = _dev_program(gpu_ctx, rp.RP_TEMPLATE_OCCUPANCY, 3, deg, den, coef, off, ow.scales, ow.hw)
    spec = rp.Spec(prog)
    s_out = spec_select(spec, 1, n_grid, cand, rp.RP_SELECT_MAX)
    t_out = table_select(prog, n_grid, cand, rp.RP_SELECT_MAX)
    compare(s_out, t_out, "occupancy")
    np.testing.assert_array_equal(s_out[0], t_out[0])
    np.testing.assert_array_equal(s_out[1], t_out[1])


@pytest.mark.parametrize("v", [1, 2, 3, 4])
def test_specialised_single_programs(gpu_ctx, orc, v):
    """40 fitted single-rational programs, candidates over v - 1 program
    parameters, both senses."""
    batch = W.uniform_batch(40, 200, v, 2, 0.0, seed=40 + v)
    coefs = [planted_in_order(orc, p) for p in batch.planted]
    coef = np.concatenate(coefs)
    off = np.zeros(41, np.int64)
    np.cumsum([len(c) for c in coefs], out=off[1:])
    deg = np.full(40, 2, np.int32)
    if v == 1:
        cand = np.zeros((1, 0), np.int32)
    else:
        g = {2: np.arange(1, 257), 3: np.arange(1, 33), 4: np.arange(1, 9)}[v]
        mesh = np.meshgrid(*([g] * (v - 1)), indexing="ij")
        cand = np.stack([a.ravel() for a in mesh], axis=-1).astype(np.int32)
    scale = [4096.0] + [float(cand.max()) if v > 1 else 1.0] * (v - 1)
    n_grid = np.array([512.0, 1024.0, 3000.0, 4096.0])
    prog = _dev_program(gpu_ctx, rp.RP_TEMPLATE_SINGLE, v, deg, deg, coef, off, scale, P=40)
    spec = rp.Spec(prog)
    for sense in (rp.RP_SELECT_MIN, rp.RP_SELECT_MAX):
        s_out = spec_select(spec, 40, n_grid, cand, sense)
        t_out = table_select(prog, n_grid, cand, sense)
        compare(s_out, t_out, f"single v={v} sense={sense}")
    oprog = orc.Program(orc.TEMPLATE_SINGLE, v, deg, deg, coef, off, scale=scale, num_programs=40)
    s_out = spec_select(spec, 40, n_grid, cand, rp.RP_SELECT_MIN)
    oam, obest, osecond = orc.argmin(oprog, n_grid, cand)
    for p in range(0, 40, 5):
        check_selection(oprog, p, n_grid, cand, s_out[0], s_out[1], oam, obest, osecond)


def test_specialised_rejects_too_many_programs(gpu_ctx, orc):
    E = orc.monomials(2, 1)
    P = 257
    coef = np.tile(np.array([1.0, 0.0, 0.0, 0.0, 0.0]), P)
    off = np.arange(P + 1, dtype=np.int64) * 5
    deg = np.ones(P, np.int32)
    prog = _dev_program(gpu_ctx, rp.RP_TEMPLATE_SINGLE, 2, deg, deg, coef, off, [1.0, 1.0], P=P)
    with pytest.raises(rp.RpError, match="256"):
        rp.Spec(prog)
