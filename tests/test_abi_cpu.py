"""Host-side checks of the C-ABI library (no GPU needed).

The library must load, export every entry point that include/rp.h declares,
produce host tables bit-identical to the oracle's, and reject bad arguments
before touching a device.
"""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

from paper_1906_00142_amd import rp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rp.h")


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(rp.LIB_PATH):
        import paper_1906_00142_amd.build as b
        b.build(verbose=False)
    return rp.lib()


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|const char\s*\*)\s+(rp_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_binding_exports():
    assert declared_symbols() == sorted(rp.EXPORTS)


def test_library_exports_every_declared_symbol(L):
    for name in declared_symbols():
        assert hasattr(L, name), name


def test_monomial_box_bit_exact_vs_oracle(L, orc):
    rng = np.random.default_rng(3)
    boxes = [[0], [5], [2, 1], [1, 2], [3, 3], [2, 0, 1], [1, 1, 1, 1], [4, 2, 3, 1],
             [15, 1], [2, 2, 2, 2, 2, 2]]
    boxes += [list(rng.integers(0, 5, size=int(rng.integers(1, 6)))) for _ in range(20)]
    for box in boxes:
        np.testing.assert_array_equal(rp.rp_monomials_box(box), orc.monomials_box(box))
    cnt = C.c_int(0)
    bad = np.array([2, 16], dtype=np.int32)
    assert L.rp_monomials_box(2, bad.ctypes.data_as(C.c_void_p), None, C.byref(cnt)) == rp.RP_EINVAL
    assert L.rp_monomials_box(0, bad.ctypes.data_as(C.c_void_p), None, C.byref(cnt)) == rp.RP_EINVAL


@pytest.mark.parametrize("v", range(1, 9))
def test_monomials_bit_exact_vs_oracle(L, orc, v):
    for d in range(0, 7 if v <= 4 else 4):
        np.testing.assert_array_equal(rp.rp_monomials(v, d), orc.monomials(v, d))
        assert len(rp.rp_monomials(v, d)) == math.comb(v + d, d)


def test_num_coefs(L, orc):
    for v in range(1, 5):
        for dn in range(0, 5):
            for dq in range(0, 5):
                assert rp.rp_num_coefs(v, dn, dq) == orc.num_coefs(v, dn, dq)


@pytest.mark.parametrize("max_prod,multiple", [(1024, 64), (1024, 32), (512, 1), (1, 1),
                                               (4096, 96), (1000, 7)])
def test_candidates_bit_exact_vs_oracle(L, orc, max_prod, multiple):
    np.testing.assert_array_equal(rp.rp_candidates_2d(max_prod, multiple),
                                  orc.candidates_2d(max_prod, multiple))


def test_argument_errors(L):
    cnt = C.c_int(0)
    assert L.rp_monomials(0, 2, None, C.byref(cnt)) == rp.RP_EINVAL
    assert b"nvars" in L.rp_last_error()
    assert L.rp_monomials(9, 2, None, C.byref(cnt)) == rp.RP_EINVAL
    assert L.rp_monomials(3, 16, None, C.byref(cnt)) == rp.RP_EINVAL
    assert L.rp_monomials(3, 2, None, None) == rp.RP_EINVAL
    assert L.rp_candidates_2d(0, 64, None, C.byref(cnt)) == rp.RP_EINVAL
    assert L.rp_num_coefs(3, -1, 2, C.byref(cnt)) == rp.RP_EINVAL
    # every handle-taking entry point rejects NULL handles before any device work
    assert L.rp_plan_create(None, 1, None, None, None, None, None) == rp.RP_EINVAL
    assert L.rp_fit_rational(None, None, 0, None, None, None, None, None, None, None) == rp.RP_EINVAL
    assert L.rp_refine_rational(None, None, 0, None, None, None, None, None, None) == rp.RP_EINVAL
    assert L.rp_loss_grad(None, None, 0, None, None, None, None, None, 0, None) == rp.RP_EINVAL
    assert L.rp_assemble_design(None, None, 0, None, 0, None, None, None) == rp.RP_EINVAL
    assert L.rp_eval_program_argmin(None, None, 0, None, 0, 0, 0, None, None, None, None,
                                    None) == rp.RP_EINVAL
    assert L.rp_program_create(None, None, None) == rp.RP_EINVAL
    assert L.rp_create(None, 0) == rp.RP_EINVAL
    assert L.rp_plan_destroy(None) == rp.RP_OK and L.rp_program_destroy(None) == rp.RP_OK


def test_missing_library_fails_loudly(monkeypatch):
    monkeypatch.setattr(rp, "LIB_PATH", "/nonexistent/librpfit.so")
    monkeypatch.setattr(rp, "_lib", None)
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        rp.lib()


def test_generated_evaluator_source_compiles_for_gfx950():
    """Code generation is host logic: the specialised evaluator's source for
    the MWP-CWP workload and for a batch of single rationals compiles with
    hipRTC for gfx950 (no device needed)."""
    import ctypes as C

    import numpy as np

    from paper_1906_00142_amd import rp
    from paper_1906_00142_amd import workloads as W
    try:
        rtc = C.CDLL("libhiprtc.so")
    except OSError:
        rtc = C.CDLL("/opt/rocm/lib/libhiprtc.so")
    pw = W.program_workload()
    coefs = [rp.planted_coefs(m) for m in pw.metrics]
    off = np.zeros(17, np.int64)
    np.cumsum([len(c) for c in coefs], out=off[1:])
    deg = np.array([m.deg_num for m in pw.metrics], np.int32)
    den = np.array([m.deg_den for m in pw.metrics], np.int32)
    sources = [rp.program_source(rp.RP_TEMPLATE_MWPCWP, 3, deg, den, off, np.concatenate(coefs),
                                 pw.scales, pw.hw)]
    b = W.uniform_batch(3, 50, 2, 3, 0.0, seed=2)
    cs = [rp.planted_coefs(p) for p in b.planted]
    o = np.zeros(4, np.int64)
    np.cumsum([len(c) for c in cs], out=o[1:])
    sources.append(rp.program_source(rp.RP_TEMPLATE_SINGLE, 2, [3] * 3, [3] * 3, o, np.concatenate(cs),
                                     [4096.0, 1024.0], num_programs=3))
    assert "case 2:" in sources[1] and "mwpcwp_cycles<double>" in sources[0]
    # coefficients appear as literals that read back exactly
    assert repr(float(cs[2][0])).rstrip("0") in sources[1] or ("%.17g" % cs[2][0]) in sources[1]
    for src in sources:
        prg = C.c_void_p()
        assert rtc.hiprtcCreateProgram(C.byref(prg), src.encode(), b"spec.hip", 0, None, None) == 0
        opts = (C.c_char_p * 4)(b"--offload-arch=gfx950", b"-O3", b"-ffp-contract=fast", b"-std=c++17")
        rc = rtc.hiprtcCompileProgram(prg, 4, opts)
        n = C.c_size_t(0)
        rtc.hiprtcGetProgramLogSize(prg, C.byref(n))
        log = C.create_string_buffer(n.value + 1)
        rtc.hiprtcGetProgramLog(prg, log)
        rtc.hiprtcDestroyProgram(C.byref(prg))
        assert rc == 0, log.value.decode()[:2000]


def _moment_tables():
    """The committed moment-group tables, parsed: {(v, code, gn): dict}."""
    path = os.path.join(ROOT, "paper_1906_00142_amd", "csrc", "rp_moment_groups.inc")
    text = open(path).read()
    out = {}
    for m in re.finditer(r"struct MomGroups<(\d+), (\d+), (true|false)> \{(.*?)\n\};", text, flags=re.S):
        body = m.group(4)
        nwv, ng, pl = (int(x) for x in re.search(r"kNWV = (\d+), kNG = (\d+), kPL = (\d+)", body).groups())
        arrays = {}
        for name in ("kPair", "kOrder", "kSlot"):
            txt = re.search(name + r"(?:\[\d+\])+ = (\{.*?\});", body, flags=re.S).group(1)
            arrays[name] = [int(x) for x in re.findall(r"-?\d+", txt)]
        out[(int(m.group(1)), int(m.group(2)), m.group(3) == "true")] = dict(nwv=nwv, ng=ng, pl=pl, **arrays)
    return out


def test_moment_group_tables_cover_every_pair_once():
    """Every compiled shape has a table for both moment Grams; its waves hold
    each moment-weight pair exactly once, kSlot inverts kPair, the variable
    orders are permutations, and the group counts are those the kernels'
    moment layout derives from the pair count."""
    shapes = [(v, d, d) for v in range(1, 5) for d in range(1, 5)] + \
             [(v, dn, dq) for v in range(1, 4) for dn, dq in ((1, 2), (2, 1), (2, 3), (3, 2))]
    tabs = _moment_tables()
    assert len(tabs) == 2 * len(shapes)
    for v, dn, dq in shapes:
        code = dn if dn == dq else dn | (dq << 4)
        dm = max(dn, dq)
        nm1, nm2 = math.comb(v + dm, dm), math.comb(v + 2 * dm, 2 * dm)
        for gn in (False, True):
            t = tabs[(v, code, gn)]
            # bands of exponents: e = 0, degree 1 (v of them), degree 2..dm, above
            npair = (3 + 4 * v + 5 * (nm1 - 1 - v) if gn else 3 * nm1) + 3 * (nm2 - nm1)
            nwv = 4 if npair <= 300 else 8
            plmax = (64 if npair <= 256 else 75) if nwv == 4 else 40
            ng = -(-(-(-npair // plmax)) // nwv) * nwv
            assert (t["nwv"], t["ng"], t["pl"]) == (nwv, ng, -(-npair // ng)), (v, dn, dq, gn)
            pairs = t["kPair"]
            assert len(pairs) == t["ng"] * t["pl"]
            used = [p for p in pairs if p >= 0]
            assert sorted(used) == list(range(npair))
            slot = t["kSlot"]
            assert len(slot) == npair and all(pairs[slot[p]] == p for p in range(npair))
            orders = np.array(t["kOrder"]).reshape(t["ng"], v)
            assert all(sorted(o) == list(range(v)) for o in orders.tolist())
