"""Writes rp_moment_groups.inc: which moment-weight pairs each wave of the
FP64 moment Gram kernels accumulates, for every compiled model shape.

Every Gram entry of a monomial design is a weighted moment sum_i w(i) m_e(u_i)
(e of total degree <= 2 DM; three weights for the linear problem, up to six
for the Jacobian, each exponent carrying only the weights its Gram entries
use), and a workgroup's waves split the moment-weight pairs between them.  A wave builds each monomial of its pairs per sample from power tables
(u_k^t) by a left-to-right product over the variables, the products of equal
leading factors shared; its cost per sample is one FMA per pair plus those
multiplies.  This script assigns the pairs to the waves (all weights of an
exponent together where they fit) so that, within each pass of NWV waves
that run between the same barriers, the costliest wave is as cheap as
possible, and picks each wave's variable order; a deterministic greedy start
is improved by a seeded local search.  Run from this directory:
python gen_moment_groups.py
"""
import itertools
import math
import random

# Shapes compiled by the library: equal degrees 1..4 in 1..4 variables, and
# degrees differing by one up to 3 in 1..3 variables (rp_internal.h).
SHAPES = [(v, d, d) for v in range(1, 5) for d in range(1, 5)] + \
         [(v, dn, dq) for v in range(1, 4) for dn, dq in ((1, 2), (2, 1), (2, 3), (3, 2))]


def graded(v, d):
    """Exponents of total degree <= d in the library's order: lower degree
    first; within a degree the larger exponent of x1 first, then of x2..."""
    out = []

    def rec(k, r, pre):
        if k == v - 1:
            out.append(tuple(pre + [r]))
            return
        for a in range(r, -1, -1):
            rec(k + 1, r - a, pre + [a])

    for t in range(d + 1):
        rec(0, t, [])
    return out


def deg_code(dn, dq):
    return dn if dn == dq else dn | (dq << 4)


class Shape:
    """The moment layout of MomentShape in rp_internal.h."""

    def __init__(self, v, dn, dq, gn):
        self.v, self.gn = v, gn
        dm = max(dn, dq)
        self.E = graded(v, 2 * dm)
        self.nm1 = math.comb(v + dm, dm)
        # weights per band of exponents (MomentPairs in rp_internal.h): e = 0,
        # degree 1 (indices 1..v in graded order), degree 2..dm, above
        z, ow, lw = (3, 4, 5) if gn else (3, 3, 3)
        self.z, self.ow, self.lw = z, ow, lw
        self.nw = [z if i == 0 else (ow if i <= v else (lw if i < self.nm1 else 3)) for i in range(len(self.E))]
        self.npair = sum(self.nw)
        self.nwv = 4 if self.npair <= 4 * 75 else 8
        plmax = (64 if self.npair <= 4 * 64 else 75) if self.nwv == 4 else 40
        ng0 = -(-self.npair // plmax)
        self.ng = -(-ng0 // self.nwv) * self.nwv
        self.pl = -(-self.npair // self.ng)

    def pair_index(self, i, w):
        """Index of exponent i's w-th pair (w a slot of i's band)."""
        v = self.v
        if i == 0:
            return w
        if i <= v:
            return self.z + (i - 1) * self.ow + w
        if i < self.nm1:
            return self.z + v * self.ow + (i - 1 - v) * self.lw + w
        return self.z + v * self.ow + (self.nm1 - 1 - v) * self.lw + (i - self.nm1) * 3 + w


def mul_cost(exps, order, v):
    """Multiplies that form the monomials of `exps` (indices into E as
    exponent tuples) in variable order `order`: the power tables up to each
    variable's largest exponent, then one multiply per distinct prefix of two
    or more nonzero factors."""
    pw = 0
    for k in range(v):
        top = max((e[k] for e in exps), default=0)
        pw += max(0, top - 1)
    pref = set()
    for e in exps:
        nz = [(k, e[k]) for k in order if e[k] > 0]
        for j in range(2, len(nz) + 1):
            pref.add(tuple(nz[:j]))
    return pw + len(pref)


class Assign:
    """Pairs (exponent index, weight) assigned to groups of at most PL."""

    def __init__(self, S):
        self.S = S
        self.orders = list(itertools.permutations(range(S.v)))
        self.groups = [[] for _ in range(S.ng)]   # lists of (i, w)
        self.cost = [0] * S.ng
        self.memo = {}

    def group_cost(self, pairs):
        key = frozenset(i for i, _ in pairs)
        if key not in self.memo:
            exps = [self.S.E[i] for i in key]
            self.memo[key] = min(mul_cost(exps, o, self.S.v) for o in self.orders)
        return len(pairs) + self.memo[key]

    def best_order(self, g):
        exps = [self.S.E[i] for i in sorted({i for i, _ in self.groups[g]})]
        return min(self.orders, key=lambda o: (mul_cost(exps, o, self.S.v), o))

    def objective(self):
        nwv = self.S.nwv
        passes = [max(self.cost[q * nwv:(q + 1) * nwv]) for q in range(self.S.ng // nwv)]
        return (sum(passes), sum(self.cost))

    def greedy(self):
        """Heaviest exponents first, all weights of one exponent into the
        group where it costs least; an exponent that fits nowhere whole is
        split, weight by weight."""
        S = self.S
        for i in sorted(range(len(S.E)), key=lambda i: (-sum(S.E[i]), -S.nw[i], i)):
            ws = [(i, w) for w in range(S.nw[i])]
            best = None
            for g in range(S.ng):
                if len(self.groups[g]) + len(ws) > S.pl:
                    continue
                c = self.group_cost(self.groups[g] + ws)
                key = (c, len(self.groups[g]), g)
                if best is None or key < best[0]:
                    best = (key, g, c)
            if best is not None:
                _, g, c = best
                self.groups[g] += ws
                self.cost[g] = c
                continue
            for pw in ws:
                cands = [g for g in range(S.ng) if len(self.groups[g]) < S.pl]
                g = min(cands, key=lambda g: (self.group_cost(self.groups[g] + [pw]), g))
                self.groups[g].append(pw)
                self.cost[g] = self.group_cost(self.groups[g])

    def improve(self, iters, seed):
        """Moves and swaps of single pairs or of all of a group's pairs of one
        exponent, kept when the objective does not get worse."""
        S = self.S
        rnd = random.Random(seed)
        cur = self.objective()
        for _ in range(iters):
            g1, g2 = rnd.randrange(S.ng), rnd.randrange(S.ng)
            if g1 == g2 or not self.groups[g1]:
                continue
            pick = self.groups[g1][rnd.randrange(len(self.groups[g1]))]
            if rnd.random() < 0.7:   # every weight of that exponent in g1
                mv = [q for q in self.groups[g1] if q[0] == pick[0]]
            else:
                mv = [pick]
            back = []
            if self.groups[g2] and rnd.random() < 0.5:
                other = self.groups[g2][rnd.randrange(len(self.groups[g2]))]
                back = [q for q in self.groups[g2] if q[0] == other[0]]
            n1 = [q for q in self.groups[g1] if q not in mv] + back
            n2 = [q for q in self.groups[g2] if q not in back] + mv
            if len(n1) > S.pl or len(n2) > S.pl:
                continue
            old = (self.groups[g1], self.groups[g2], self.cost[g1], self.cost[g2])
            self.groups[g1], self.groups[g2] = n1, n2
            self.cost[g1], self.cost[g2] = self.group_cost(n1), self.group_cost(n2)
            new = self.objective()
            if new <= cur:
                cur = new
            else:
                self.groups[g1], self.groups[g2], self.cost[g1], self.cost[g2] = old
        return cur


def index_order_objective(S):
    """The same objective for the pairs taken in index order, PL per wave."""
    pairs = [(i, w) for i in range(len(S.E)) for w in range(S.nw[i])]
    A = Assign(S)
    for g in range(S.ng):
        grp = pairs[g * S.pl:(g + 1) * S.pl]
        A.groups[g] = grp
        A.cost[g] = len(grp) + mul_cost([S.E[i] for i in sorted({i for i, _ in grp})],
                                        tuple(range(S.v)), S.v)
    return A.objective()


def table(v, dn, dq, gn, iters=3000):
    S = Shape(v, dn, dq, gn)
    A = Assign(S)
    A.greedy()
    A.improve(iters * S.ng, seed=1906 + 131 * v + 17 * dn + 5 * dq + int(gn))
    rows, orders = [], []
    for g in range(S.ng):
        ps = sorted(S.pair_index(i, w) for i, w in A.groups[g])
        rows.append(ps + [-1] * (S.pl - len(ps)))
        orders.append(list(A.best_order(g)))
    slot = [0] * S.npair
    for g, r in enumerate(rows):
        for j, p in enumerate(r):
            if p >= 0:
                slot[p] = g * S.pl + j
    assert sorted(p for r in rows for p in r if p >= 0) == list(range(S.npair))
    return (rows, orders, slot), S, A.objective()


def arr(a):
    return "{" + ", ".join(map(str, a)) + "}"


def main():
    out = ["// Generated by gen_moment_groups.py: the moment-weight pairs of each wave",
           "// of the FP64 moment Gram kernels (kPair[group][slot], -1 = unused slot),",
           "// each wave's variable order for forming its monomials, and the slot of",
           "// every pair (kSlot[pair]).  Per-sample cost per pass (FMAs + multiplies",
           "// of the costliest wave, summed over passes): index order -> this table.",
           ""]
    for v, dn, dq in SHAPES:
        for gn in (False, True):
            t, S, obj = table(v, dn, dq, gn)
            name = f"MomGroups<{v}, {deg_code(dn, dq)}, {'true' if gn else 'false'}>"
            rows, orders, slot = t
            base = index_order_objective(S)
            out.append(f"// {v} variables, degree {dn}/{dq}, {'Jacobian' if gn else 'linear'}: "
                       f"{S.npair} pairs, {S.ng} waves of <= {S.pl}; cost {base[0]} -> {obj[0]}")
            out.append(f"template <> struct {name} {{")
            out.append("  static constexpr bool kHas = true;")
            out.append(f"  static constexpr int kNWV = {S.nwv}, kNG = {S.ng}, kPL = {S.pl};")
            out.append(f"  static constexpr int kPair[{S.ng}][{S.pl}] = {{{', '.join(arr(r) for r in rows)}}};")
            out.append(f"  static constexpr int kOrder[{S.ng}][{v}] = {{{', '.join(arr(o) for o in orders)}}};")
            out.append(f"  static constexpr int kSlot[{S.npair}] = {arr(slot)};")
            out.append("};")
            print(name, "cost", base[0], "->", obj[0], flush=True)
    with open("rp_moment_groups.inc", "w") as f:
        f.write("\n".join(out) + "\n")


if __name__ == "__main__":
    main()
