"""Helpers of the GPU parity tests (test code: plain NumPy on the oracle's
exponent tables and evaluator)."""
import numpy as np

# predictions are compared where the oracle's |Q| is at least this: near a
# root of Q the prediction N/Q is unbounded and says nothing about the fit
Q_FLOOR = 1e-3


def q_values(orc, u, coef, v, dn, dq):
    """Q at the samples u[k, i] from the oracle's exponent table (plain
    products of the variables, no powers)."""
    na = len(orc.monomials(v, dn))
    E = orc.monomials(v, dq).astype(np.int64)[1:]
    beta = coef[na:]
    pw = [[np.ones(u.shape[1])] for _ in range(v)]
    for k in range(v):
        for _ in range(int(E[:, k].max()) if len(E) else 0):
            pw[k].append(pw[k][-1] * u[k])
    q = np.ones(u.shape[1])
    for j, e in enumerate(E):
        mono = pw[0][int(e[0])]
        for k in range(1, v):
            mono = mono * pw[k][int(e[k])]
        q = q + beta[j] * mono
    return q


def masked_pred_rel_err(orc, u, v, dn, dq, coef, ocoef):
    """max |f - f_oracle| / max |f_oracle| over the samples where the
    oracle's |Q| >= Q_FLOOR (0 when there is none)."""
    keep = np.abs(q_values(orc, u, ocoef, v, dn, dq)) >= Q_FLOOR
    if not keep.any():
        return 0.0
    pa = orc.eval_rational(v, dn, dq, coef, u[:, keep])
    po = orc.eval_rational(v, dn, dq, ocoef, u[:, keep])
    return float(np.max(np.abs(pa - po)) / np.max(np.abs(po)))
