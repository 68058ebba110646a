"""Seeded synthetic workloads for the rational-program hot path.

The paper collects its samples by running or emulating the tuned program
(Section 3.3, step 1; Section 4.1).  Here that step is replaced by samples of
*planted* rational functions, drawn from seeded NumPy generators, with the
shapes of the paper's setting: a data size, thread-block dimensions whose
product is a multiple of the wave size, and noisy low-level metrics.

This module only draws inputs.  It holds none of the method's arithmetic: it
does not order monomials, enumerate candidates, assemble designs, fit, or
evaluate programs.  A planted function is stored as an *unordered* list of
exponent tuples with their coefficients (in ``itertools.product`` order),
which consumers map onto the method's monomial order by tuple.  Both the GPU
path and the CPU oracle read these arrays; neither is imported here.

Seeds: workload ``k`` uses master seed ``190600142 + k`` and fit ``f`` draws
from ``numpy.random.default_rng([seed, f])``.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np

MASTER_SEED = 190600142


def seed_for(k: int) -> int:
    return MASTER_SEED + int(k)


def _exponent_tuples(nvars: int, degree: int) -> np.ndarray:
    """All exponent tuples of total degree <= degree, in itertools order."""
    rows = [e for e in itertools.product(range(degree + 1), repeat=nvars)
            if sum(e) <= degree]
    return np.asarray(rows, dtype=np.int64).reshape(-1, nvars)


@dataclass
class Planted:
    """A planted rational function N/Q with Q's constant term equal to 1."""
    nvars: int
    deg_num: int
    deg_den: int
    num_exps: np.ndarray          # [a, v] int
    num_coef: np.ndarray          # [a]
    den_exps: np.ndarray          # [b, v] int, constant tuple excluded
    den_coef: np.ndarray          # [b]

    def value(self, u: np.ndarray) -> np.ndarray:
        """Planted f(u) for u of shape [v, m] (used only to synthesise samples)."""
        u = np.asarray(u, dtype=np.float64)
        mn = np.prod(u[None, :, :] ** self.num_exps[:, :, None], axis=1)
        md = np.prod(u[None, :, :] ** self.den_exps[:, :, None], axis=1)
        return (self.num_coef @ mn) / (1.0 + self.den_coef @ md)

    def coef_by_tuple(self):
        """(numerator dict, denominator dict) keyed by exponent tuple."""
        num = {tuple(int(t) for t in e): float(c)
               for e, c in zip(self.num_exps, self.num_coef)}
        den = {tuple(int(t) for t in e): float(c)
               for e, c in zip(self.den_exps, self.den_coef)}
        return num, den


def plant(rng: np.random.Generator, nvars: int, deg_num: int, deg_den: int,
          num_lo=-1.0, num_hi=1.0, den_lo=0.0, den_hi=0.1) -> Planted:
    ne = _exponent_tuples(nvars, deg_num)
    de = _exponent_tuples(nvars, deg_den)
    de = de[de.sum(axis=1) > 0]
    nc = rng.uniform(num_lo, num_hi, size=len(ne))
    dc = rng.uniform(den_lo, den_hi, size=len(de))
    return Planted(nvars, deg_num, deg_den, ne, nc, de, dc)


@dataclass
class FitBatch:
    """An uneven batch of fits in structure-of-arrays layout.

    ``x[k, s]`` is normalised variable k of global sample s (rows k >= nvars[f]
    are zero for fit f); fit f owns samples ``sample_off[f]:sample_off[f+1]``.
    """
    num_fits: int
    max_vars: int
    sample_off: np.ndarray        # int64 [F+1]
    nvars: np.ndarray             # int32 [F]
    deg_num: np.ndarray           # int32 [F]
    deg_den: np.ndarray           # int32 [F]
    x: np.ndarray                 # float64 [max_vars, total]
    y: np.ndarray                 # float64 [total]
    noise: float
    planted: list = field(default_factory=list)
    label: str = ""

    @property
    def total_samples(self) -> int:
        return int(self.sample_off[-1])

    def fit_samples(self, f: int):
        a, b = int(self.sample_off[f]), int(self.sample_off[f + 1])
        v = int(self.nvars[f])
        return self.x[:v, a:b], self.y[a:b]


def _assemble(parts, max_vars, noise, label) -> FitBatch:
    F = len(parts)
    counts = np.array([p[1].shape[1] for p in parts], dtype=np.int64)
    off = np.zeros(F + 1, dtype=np.int64)
    np.cumsum(counts, out=off[1:])
    x = np.zeros((max_vars, int(off[-1])), dtype=np.float64)
    y = np.empty(int(off[-1]), dtype=np.float64)
    for f, (pl, u, yy) in enumerate(parts):
        x[:u.shape[0], off[f]:off[f + 1]] = u
        y[off[f]:off[f + 1]] = yy
    return FitBatch(
        num_fits=F, max_vars=max_vars, sample_off=off,
        nvars=np.array([p[0].nvars for p in parts], dtype=np.int32),
        deg_num=np.array([p[0].deg_num for p in parts], dtype=np.int32),
        deg_den=np.array([p[0].deg_den for p in parts], dtype=np.int32),
        x=x, y=y, noise=noise, planted=[p[0] for p in parts], label=label)


def _noisy(rng, pl: Planted, u: np.ndarray, sigma: float) -> np.ndarray:
    f = pl.value(u)
    if sigma == 0.0:
        return f
    return f * (1.0 + sigma * rng.standard_normal(f.shape[0]))


# ---------------------------------------------------------------------------
# Fit workloads
# ---------------------------------------------------------------------------

def tiny_fit(seed: int | None = None, sigma: float = 0.01,
             num_samples: int = 256) -> FitBatch:
    """One metric over (data size n, block size b), degree 2/2, 256 samples.

    n is log-uniform over [2^8, 2^14] and rounded to an integer; b is one of
    32, 64, ..., 1024.  Variables are normalised by their domain maxima:
    u = (n / 2^14, b / 1024).
    """
    seed = seed_for(0) if seed is None else seed
    rng = np.random.default_rng([seed, 0])
    pl = plant(rng, 2, 2, 2)
    n = np.rint(2.0 ** rng.uniform(8.0, 14.0, size=num_samples))
    b = 32.0 * rng.integers(1, 33, size=num_samples)
    u = np.stack([n / 2.0 ** 14, b / 1024.0])
    return _assemble([(pl, u, _noisy(rng, pl, u, sigma))], 2, sigma, "tiny")


def uniform_batch(num_fits: int, num_samples: int, nvars: int, degree: int,
                  sigma: float, seed: int, label: str = "", deg_den: int | None = None) -> FitBatch:
    """num_fits independent fits, u ~ U[0,1]^nvars, planted with numerator
    degree `degree` and denominator degree `deg_den` (default: the same)."""
    dq = degree if deg_den is None else deg_den
    parts = []
    for f in range(num_fits):
        rng = np.random.default_rng([seed, f])
        pl = plant(rng, nvars, degree, dq)
        u = rng.uniform(0.0, 1.0, size=(nvars, num_samples))
        parts.append((pl, u, _noisy(rng, pl, u, sigma)))
    return _assemble(parts, nvars, sigma, label)


def batched_fit(num_fits: int = 4096, num_samples: int = 2048,
                sigma: float = 0.005, seed: int | None = None) -> FitBatch:
    """4096 fits over (n, bx, by), degree 3/3 (20 + 19 unknowns), 2048 samples."""
    seed = seed_for(1) if seed is None else seed
    return uniform_batch(num_fits, num_samples, 3, 3, sigma, seed, "batched")


def refine_batch(num_fits: int = 4096, num_samples: int = 2048,
                 sigma: float = 0.005, seed: int | None = None) -> FitBatch:
    """The batched shape again, drawn from its own seed, for true-loss refinement."""
    seed = seed_for(3) if seed is None else seed
    return uniform_batch(num_fits, num_samples, 3, 3, sigma, seed, "refine")


def uneven_batch(num_fits: int = 16384, m_lo: int = 64, m_hi: int = 8192,
                 sigma: float = 0.005, seed: int | None = None,
                 nvars_choices=(2, 3, 4), deg_choices=(1, 2, 3, 4)) -> FitBatch:
    """Uneven batch: m log-uniform in [m_lo, m_hi], v and d drawn per fit."""
    seed = seed_for(4) if seed is None else seed
    lg = np.log2(m_hi / m_lo)
    parts = []
    for f in range(num_fits):
        rng = np.random.default_rng([seed, f])
        m = int(np.rint(m_lo * 2.0 ** (lg * rng.uniform())))
        v = int(rng.choice(nvars_choices))
        d = int(rng.choice(deg_choices))
        pl = plant(rng, v, d, d)
        u = rng.uniform(0.0, 1.0, size=(v, m))
        parts.append((pl, u, _noisy(rng, pl, u, sigma)))
    return _assemble(parts, max(nvars_choices), sigma, "uneven")


def interpolation_batch(num_fits: int, nvars: int, degree: int,
                        seed: int) -> FitBatch:
    """Noise-free fits whose sample count equals the number of unknowns."""
    parts = []
    for f in range(num_fits):
        rng = np.random.default_rng([seed, f])
        pl = plant(rng, nvars, degree, degree)
        n_unknowns = len(pl.num_coef) + len(pl.den_coef)
        u = rng.uniform(0.0, 1.0, size=(nvars, n_unknowns))
        parts.append((pl, u, pl.value(u)))
    return _assemble(parts, nvars, 0.0, "interp")


# ---------------------------------------------------------------------------
# Program-evaluation workloads
# ---------------------------------------------------------------------------

# Slots of the 16 low-level metrics combined by the MWP-CWP-style template.
METRIC_NAMES = (
    "comp_insts", "coal_mem_insts", "uncoal_mem_insts", "synch_insts",
    "coal_per_mw", "uncoal_per_mw", "load_bytes_per_warp", "regs_per_thread",
    "lds_bytes_per_block", "total_blocks", "sfu_insts", "lds_insts",
    "lds_conflict_rate", "branch_insts", "l2_hit_rate", "divergence_rate",
)

# Hardware vector layout (one float64 per entry).
HW_NAMES = (
    "wave_size", "num_cu", "simd_per_cu", "max_threads_per_block",
    "max_blocks_per_cu", "max_waves_per_cu", "regs_per_cu", "lds_bytes_per_cu",
    "mem_latency", "l2_latency", "departure_del_coal", "departure_del_uncoal",
    "issue_cycles", "sfu_issue_cycles", "lds_issue_cycles", "clock_ghz",
    "mem_bandwidth_gbs",
)


def hardware_vector(rng: np.random.Generator) -> np.ndarray:
    """Seeded hardware parameters: fixed MI355X-like counts, drawn latencies."""
    hw = {
        "wave_size": 64.0, "num_cu": 256.0, "simd_per_cu": 4.0,
        "max_threads_per_block": 1024.0, "max_blocks_per_cu": 32.0,
        "max_waves_per_cu": 32.0, "regs_per_cu": 4.0 * 512.0 * 64.0,
        "lds_bytes_per_cu": 163840.0,
        "mem_latency": float(np.rint(rng.uniform(400.0, 900.0))),
        "l2_latency": float(np.rint(rng.uniform(150.0, 300.0))),
        "departure_del_coal": float(np.rint(rng.uniform(2.0, 8.0))),
        "departure_del_uncoal": float(np.rint(rng.uniform(20.0, 60.0))),
        "issue_cycles": float(np.rint(rng.uniform(1.0, 4.0))),
        "sfu_issue_cycles": float(np.rint(rng.uniform(4.0, 16.0))),
        "lds_issue_cycles": float(np.rint(rng.uniform(2.0, 8.0))),
        "clock_ghz": 2.4, "mem_bandwidth_gbs": 8000.0,
    }
    return np.array([hw[k] for k in HW_NAMES], dtype=np.float64)


def _structured_metric(rng, slot: int, degree: int) -> Planted:
    """A nonnegative planted metric over u = (n/2^24, bx/1024, by/1024).

    Every monomial gets a small nonnegative coefficient; a few dominant terms
    give each slot the qualitative dependence a real kernel metric has (work per
    thread growing with n, block count falling with block size, LDS use
    growing with block size, and so on).
    """
    pl = plant(rng, 3, degree, degree, 0.0, 1.0, 0.0, 0.05)
    num = pl.num_coef
    den = pl.den_coef
    idx_n = {tuple(e): i for i, e in enumerate(pl.num_exps.tolist())}
    idx_d = {tuple(e): i for i, e in enumerate(pl.den_exps.tolist())}
    s = rng.uniform(0.5, 2.0)

    def setn(e, v):
        num[idx_n[e]] = v

    def setd(e, v):
        den[idx_d[e]] = v

    if slot == 0:        # comp_insts: grows with n
        num *= 8.0 * s; setn((0, 0, 0), 40.0 * s); setn((1, 0, 0), 4000.0 * s)
    elif slot == 1:      # coal_mem_insts
        num *= 2.0 * s; setn((0, 0, 0), 4.0 * s); setn((1, 0, 0), 600.0 * s)
        setn((0, 1, 0), 6.0 * s)
    elif slot == 2:      # uncoal_mem_insts: fall as bx grows
        num *= 1.0 * s; setn((0, 0, 0), 2.0 * s); setn((1, 0, 0), 300.0 * s)
        setd((0, 1, 0), 20.0 * s)
    elif slot == 3:      # synch_insts
        num *= 0.2 * s; setn((0, 0, 0), 1.0 * s)
    elif slot == 4:      # coal_per_mw
        num *= 0.2; setn((0, 0, 0), 1.0 + s)
    elif slot == 5:      # uncoal_per_mw: grows with by
        num *= 0.5; setn((0, 0, 0), 2.0 * s); setn((0, 0, 1), 24.0 * s)
    elif slot == 6:      # load_bytes_per_warp
        num *= 4.0; setn((0, 0, 0), 256.0 * s)
    elif slot == 7:      # regs_per_thread
        num *= 4.0; setn((0, 0, 0), 24.0 + 16.0 * s)
        setn((0, 1, 0), 8.0 * s); setn((0, 0, 1), 8.0 * s)
    elif slot == 8:      # lds_bytes_per_block: proportional to bx*by
        num *= 16.0; setn((0, 0, 0), 64.0 * s); setn((0, 1, 1), 4.0 * 1048576.0 * s)
    elif slot == 9:      # total_blocks ~ n / (bx*by)
        num *= 4.0; setn((1, 0, 0), 16777216.0 * s); setn((0, 0, 0), 8.0)
        setd((0, 1, 1), 1048576.0)
    elif slot == 10:     # sfu_insts
        num *= 1.0 * s; setn((1, 0, 0), 50.0 * s)
    elif slot == 11:     # lds_insts
        num *= 2.0 * s; setn((0, 0, 0), 8.0 * s); setn((0, 1, 0), 12.0 * s)
    elif slot == 12:     # lds_conflict_rate
        num *= 0.05; setn((0, 0, 1), 0.6 * s)
    elif slot == 13:     # branch_insts
        num *= 1.0 * s; setn((0, 0, 0), 6.0 * s); setn((1, 0, 0), 100.0 * s)
    elif slot == 14:     # l2_hit_rate in [0, 1]
        num *= 0.02; setn((0, 0, 0), 0.3 * s / 2.0); setd((1, 0, 0), 2.0 * s)
    elif slot == 15:     # divergence_rate in [0, 1]
        num *= 0.02; setn((0, 1, 0), 0.2); setd((0, 1, 0), 1.0)
    return pl


@dataclass
class ProgramWorkload:
    """Planted metric rationals, a hardware vector and the data sizes to score."""
    nvars: int
    scales: np.ndarray                # [nvars] normalisation maxima
    metrics: list                     # [L] Planted
    hw: np.ndarray                    # [len(HW_NAMES)]
    n_grid: np.ndarray                # [num_n] data sizes (integers as float64)
    label: str = ""


def program_workload(seed: int | None = None, num_n: int = 1024) -> ProgramWorkload:
    """16 metric rationals of degree 2-3 over (n, bx, by) and 1024 data sizes
    n_j = round(2^(10 + 14 j / (num_n - 1))) spanning [2^10, 2^24]."""
    seed = seed_for(2) if seed is None else seed
    rng = np.random.default_rng([seed, 0])
    metrics = []
    for slot in range(len(METRIC_NAMES)):
        d = int(rng.integers(2, 4))
        metrics.append(_structured_metric(rng, slot, d))
    hw = hardware_vector(rng)
    j = np.arange(num_n, dtype=np.float64)
    n_grid = np.rint(2.0 ** (10.0 + 14.0 * j / max(num_n - 1, 1)))
    scales = np.array([2.0 ** 24, 1024.0, 1024.0])
    return ProgramWorkload(3, scales, metrics, hw, n_grid, "program")


def occupancy_workload(pw: ProgramWorkload | None = None) -> ProgramWorkload:
    """The hardware-occupancy program of a program workload: its
    registers-per-thread and LDS-bytes-per-block metrics, hardware vector,
    data sizes and scales."""
    pw = program_workload() if pw is None else pw
    slots = (METRIC_NAMES.index("regs_per_thread"), METRIC_NAMES.index("lds_bytes_per_block"))
    return ProgramWorkload(pw.nvars, pw.scales, [pw.metrics[k] for k in slots], pw.hw, pw.n_grid,
                           "occupancy")


def tiny_grid(num_n: int = 64) -> np.ndarray:
    """Data sizes n_j = round(2^(8 + 6 j / (num_n - 1))) for the tiny workload."""
    j = np.arange(num_n, dtype=np.float64)
    return np.rint(2.0 ** (8.0 + 6.0 * j / max(num_n - 1, 1)))


# ---------------------------------------------------------------------------
# Decision-node workload
# ---------------------------------------------------------------------------

@dataclass
class SplitBatch:
    """Samples of piecewise rational functions with one decision node each:
    y = f_L(u) where u[split_var] <= theta, f_R(u) elsewhere (two planted
    rationals of the same degree), in the FitBatch layout (node f owns samples
    sample_off[f]:sample_off[f+1], all nodes of one shape and size)."""
    batch: FitBatch
    split_var: int
    theta: np.ndarray             # planted thresholds [F]
    left: list
    right: list


def split_batch(num_nodes: int = 64, num_samples: int = 256, nvars: int = 2, degree: int = 2,
                split_var: int = 0, sigma: float = 0.005, seed: int = 7,
                gap: float = 0.0) -> SplitBatch:
    """Stand-in for sampled metrics that are piecewise rational in their
    parameters (a resource limit switching the binding term): per node, two
    planted rationals (numerator U[-1, 1], denominator 1 + U[0, 0.1] terms),
    a threshold theta ~ U[0.3, 0.7] on u[split_var], u ~ U[0, 1]^nvars, with
    the samples of u[split_var] in (theta - gap, theta + gap) moved out of
    that band (gap > 0 makes the planted split unambiguous), and
    multiplicative noise sigma."""
    parts, thetas, lefts, rights = [], [], [], []
    for f in range(num_nodes):
        rng = np.random.default_rng([seed, f])
        pl = plant(rng, nvars, degree, degree)
        pr = plant(rng, nvars, degree, degree)
        th = float(rng.uniform(0.3, 0.7))
        u = rng.uniform(0.0, 1.0, size=(nvars, num_samples))
        if gap > 0.0:
            s = u[split_var]
            band = np.abs(s - th) < gap
            u[split_var, band] = np.where(s[band] < th, th - gap - 0.5 * gap * rng.uniform(size=band.sum()),
                                          th + gap + 0.5 * gap * rng.uniform(size=band.sum()))
        left = u[split_var] <= th
        yl = _noisy(rng, pl, u, sigma)
        yr = _noisy(rng, pr, u, sigma)
        parts.append((pl, u, np.where(left, yl, yr)))
        thetas.append(th)
        lefts.append(pl)
        rights.append(pr)
    b = _assemble(parts, nvars, sigma, "split")
    return SplitBatch(b, split_var, np.array(thetas), lefts, rights)
