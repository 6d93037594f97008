"""Fuzzy C-Means in exact or high-precision arithmetic, for tiny inputs (test infrastructure only).

For m = 2 and m = 3 every quantity of Eq.1, Eq.3 and Eq.4 is a rational
function of the data and the initial centroids (the exponent 2/(m-1) is 2 or
1, and u^m is an integer power), so the iteration of Algorithm 1 can be run in
exact rational arithmetic.  For other m it runs in 60-digit decimal
arithmetic.  Either way the result is the exact trajectory to far below FP64
rounding, which pins the FP64 modules on small cases.
"""
from __future__ import annotations

import decimal
from fractions import Fraction


def solve_rational(x, v0, m: int, iters: int):
    """Exact trajectory for integer m in {2, 3}: returns (vs, deltas, Js) as Fractions."""
    assert m in (2, 3)
    e = Fraction(2, m - 1)
    assert e.denominator == 1
    e = int(e)
    xs = [Fraction(int(a)) for a in x]
    v = [Fraction(b) for b in v0]
    C = len(v)

    def memb(v):
        out = []
        for xi in xs:
            d = [abs(xi - vk) for vk in v]
            zeros = [k for k in range(C) if d[k] == 0]
            if zeros:
                out.append([Fraction(1, len(zeros)) if k in zeros else Fraction(0) for k in range(C)])
                continue
            out.append([1 / sum((d[j] / d[k]) ** e for k in range(C)) for j in range(C)])
        return out

    def J(U, v):
        return sum(U[i][j] ** m * (xs[i] - v[j]) ** 2 for i in range(len(xs)) for j in range(C))

    U = memb(v)
    vs, ds, Js = [list(v)], [None], [J(U, v)]
    for _ in range(iters):
        newv = []
        for j in range(C):
            den = sum(U[i][j] ** m for i in range(len(xs)))
            num = sum(U[i][j] ** m * xs[i] for i in range(len(xs)))
            newv.append(num / den if den != 0 else v[j])
        v = newv
        U2 = memb(v)
        ds.append(max(abs(U2[i][j] - U[i][j]) for i in range(len(xs)) for j in range(C)))
        U = U2
        vs.append(list(v))
        Js.append(J(U, v))
    return vs, ds, Js


def solve_decimal(x, v0, m, iters: int, digits: int = 60):
    """Trajectory in ``digits``-digit decimal arithmetic for any m > 1."""
    ctx = decimal.Context(prec=digits)
    D = ctx.create_decimal
    with decimal.localcontext(ctx):
        xs = [D(int(a)) for a in x]
        v = [D(repr(float(b))) if not isinstance(b, decimal.Decimal) else b for b in v0]
        mm = D(repr(float(m)))
        e = D(2) / (mm - 1)
        C = len(v)

        def memb(v):
            out = []
            for xi in xs:
                d = [abs(xi - vk) for vk in v]
                zeros = [k for k in range(C) if d[k] == 0]
                if zeros:
                    out.append([D(1) / len(zeros) if k in zeros else D(0) for k in range(C)])
                    continue
                out.append([D(1) / sum((d[j] / d[k]) ** e for k in range(C)) for j in range(C)])
            return out

        def powm(u):
            return u ** mm if u != 0 else D(0)

        def J(U, v):
            return sum(powm(U[i][j]) * (xs[i] - v[j]) ** 2 for i in range(len(xs)) for j in range(C))

        U = memb(v)
        vs, ds, Js = [list(v)], [None], [J(U, v)]
        for _ in range(iters):
            newv = []
            for j in range(C):
                a = [powm(U[i][j]) for i in range(len(xs))]
                den = sum(a)
                num = sum(ai * xi for ai, xi in zip(a, xs))
                newv.append(num / den if den != 0 else v[j])
            v = newv
            U2 = memb(v)
            ds.append(max(abs(U2[i][j] - U[i][j]) for i in range(len(xs)) for j in range(C)))
            U = U2
            vs.append(list(v))
            Js.append(J(U, v))
    return vs, ds, Js


def step_rational(x, v, m: int):
    """One exact step of Algorithm 1 from centroids ``v`` (any rationals):
    returns (v_next, delta, J_next) with U = memb(v), v_next = cent(U),
    delta = max |memb(v_next) - U| and J_next = J(memb(v_next), v_next)."""
    vs, ds, Js = solve_rational(x, [Fraction(a) for a in v], m, 1)
    return vs[1], ds[1], Js[1]
