"""Shared test helpers (not collected)."""
import numpy as np


def tt_substitute(ops, cuts):
    """Replace every T by T T (= S): returns the non-Clifford op list with
    its cut list re-indexed, and the equivalent Clifford op list (S in place
    of each T T)."""
    out, cl, idx = [], [], {}
    for i, op in enumerate(ops):
        if op[0] == "T":
            out += [op, op]
            cl.append(("S", op[1], -1, 0.0))
        else:
            out.append(op)
            cl.append(op)
        idx[i] = len(out) - 1
    return out, [(q, idx[a]) for q, a in cuts], cl


def stabilizer_rows(n, ops):
    from oracle import chp
    t = chp.Tableau(n)
    for k, a, b, _ in ops:
        t.gate(k, a, b)
    x, z, r = t.dump()
    return x[n:2 * n], z[n:2 * n], r[n:2 * n]
