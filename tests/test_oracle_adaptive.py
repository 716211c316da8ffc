"""Pins for the oracle's controlled-step push (Sec. 1, Sec. 2.1: fifth-order
Runge-Kutta with a controlled step, run until the kinetic energy is constant).

Independent checks: the embedded pair satisfies the order conditions of
every rooted tree up to order 5 (fifth-order weights) and 4 (embedded
weights), computed here from the trees; hyperbolic motion in a uniform field
(closed form); the focused-field solution agrees with a fine fixed-step RK4
solution of the same equations; the error falls with the tolerance; the early
stop leaves the energy within the stated tolerance of the full-window one;
the step budget is enforced.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

C = 299792458.0
QE = 1.602176634e-19
ME = 9.1093837015e-31


def _trees(order):
    """Rooted trees with `order` nodes as sorted tuples of subtrees."""
    if order == 1:
        return [()]
    out = set()

    def partitions(n, max_part):
        if n == 0:
            yield []
            return
        for p in range(min(n, max_part), 0, -1):
            for rest in partitions(n - p, p):
                yield [p] + rest

    for parts in partitions(order - 1, order - 1):
        def combos(i):
            if i == len(parts):
                yield []
                return
            for t in _trees(parts[i]):
                for rest in combos(i + 1):
                    yield [t] + rest
        for c in combos(0):
            out.add(tuple(sorted(c)))
    return sorted(out)


def _size(t):
    return 1 + sum(_size(s) for s in t)


def _density(t):
    return _size(t) * math.prod(_density(s) for s in t)


def _phi(t, A):
    """Elementary weight vector of tree t for stage matrix A (exact fractions)."""
    n = len(A)
    v = [Fraction(1)] * n
    for s in t:
        w = _phi(s, A)
        aw = [sum(A[i][j] * w[j] for j in range(n)) for i in range(n)]
        v = [v[i] * aw[i] for i in range(n)]
    return v


def test_pair_order_conditions(orc):
    c, a, b5, b4 = orc.dp_tableau()
    A = [[Fraction(x).limit_denominator(10 ** 7) for x in row] for row in a]
    F = lambda v: [Fraction(x).limit_denominator(10 ** 7) for x in v]
    b5, b4, cc = F(b5), F(b4), F(c)
    # the fractions recovered are the doubles' values to within rounding
    assert all(abs(float(A[i][j]) - a[i][j]) <= 1e-15 * max(1, abs(a[i][j]))
               for i in range(7) for j in range(7))
    for i in range(7):
        assert sum(A[i]) == cc[i]                       # row sums are the nodes
    counts = {q: len(_trees(q)) for q in range(1, 6)}
    assert counts == {1: 1, 2: 1, 3: 2, 4: 4, 5: 9}
    for q in range(1, 6):
        for t in _trees(q):
            phi = _phi(t, A)
            assert sum(b5[i] * phi[i] for i in range(7)) == Fraction(1, _density(t)), (q, t)
            if q <= 4:
                assert sum(b4[i] * phi[i] for i in range(7)) == Fraction(1, _density(t)), (q, t)
    # the embedded weights are not of fifth order (the pair has an error estimate)
    assert any(sum(b4[i] * _phi(t, A)[i] for i in range(7)) != Fraction(1, _density(t))
               for t in _trees(5))
    # first same as last: the last stage sits at the fifth-order result
    assert A[6] == b5[:6] + [Fraction(0)] or A[6][:6] == b5[:6]


def test_uniform_field_hyperbolic_motion(orc):
    E0 = 1e12
    L = orc.laser_intensity(0.8e-6, 3e-6, 30e-15, 1e21, field=orc.UNIFORM_EB,
                            test_E=(E0, 0, 0), window=1)
    A = orc.adaptive(L=L, k_tol=0.0)
    T = 100e-15
    xf, uf, ts, na, nr, st = orc.push_one_adaptive(L, A, 0.0, T, np.zeros(3), np.zeros(3))
    a = QE * E0 / (ME * C)
    assert st == 0 and ts == T and nr == 0
    assert abs(uf[0] / (-a * T) - 1) < 1e-13 and uf[1] == 0 and uf[2] == 0
    dx = -(ME * C ** 2 / (QE * E0)) * (math.sqrt(1 + (a * T) ** 2) - 1)
    assert abs(xf[0] / dx - 1) < 1e-12
    # smooth problem: first step dt, growth of at most x5 per step, then steps at
    # the cap h_max = 10 dt (the growth may take a step or two longer)
    assert 0 <= na - (2 + math.ceil((T - 6 * L.dt) / A.h_max - 1e-9)) <= 2


def test_focused_field_agrees_with_fine_rk4(orc):
    L = orc.laser_intensity(0.8e-6, 3e-6, 30e-15, 1e21)
    A = orc.adaptive(rtol=1e-11, atol=1e-11, L=L, k_tol=0.0)
    for x0, z0 in ((1e-6, 0.0), (2.5e-6, 6e-6), (0.3e-6, -4e-6)):
        t0, t1 = z0 / C - 15e-15, z0 / C + 120e-15
        X0 = np.array([x0, 0.4e-6, z0])
        xf, uf, ts, na, nr, st = orc.push_one_adaptive(L, A, t0, t1, X0, np.zeros(3))
        rx, ru = orc.push_one(L, t0, t1, L.dt / 10, X0, np.zeros(3))
        g, gr = math.sqrt(1 + uf @ uf), math.sqrt(1 + ru @ ru)
        assert st == 0 and ts == t1
        assert abs(g / gr - 1) < 1e-9, (g, gr)
        assert np.max(np.abs(uf - ru)) < 1e-8 * max(1.0, np.max(np.abs(ru)))
        assert np.max(np.abs(xf - rx)) < 1e-9 * max(L.lambda_, np.max(np.abs(rx)))


def test_error_falls_with_tolerance(orc):
    L = orc.laser_intensity(0.8e-6, 3e-6, 30e-15, 1e21)
    t0, t1 = -15e-15, 120e-15
    X0 = np.array([1.2e-6, 0.0, 0.0])
    ref = orc.push_one_adaptive(L, orc.adaptive(rtol=1e-13, atol=1e-13, L=L, k_tol=0.0), t0, t1,
                                X0, np.zeros(3))[1]
    errs, steps = [], []
    for tol in (1e-6, 1e-8, 1e-10):
        r = orc.push_one_adaptive(L, orc.adaptive(rtol=tol, atol=tol, h_max=1e-15, L=L, k_tol=0.0),
                                  t0, t1, X0, np.zeros(3))
        errs.append(np.max(np.abs(r[1] - ref)) / np.max(np.abs(ref)))
        steps.append(r[3])
    assert errs[0] > errs[1] > errs[2]
    assert errs[1] < 1e-6 and errs[2] < 1e-8
    assert steps[0] < steps[1] < steps[2]


def test_early_stop_when_energy_constant(orc):
    L = orc.laser_intensity(0.8e-6, 3e-6, 30e-15, 1e18)
    X0 = np.array([2e-6, 0.5e-6, 0.0])
    full = orc.push_one_adaptive(L, orc.adaptive(L=L, k_tol=-1.0), -10e-15, 1000e-15, X0,
                                 np.zeros(3))
    early = orc.push_one_adaptive(L, orc.adaptive(L=L, k_tol=1e-10), -10e-15, 1000e-15, X0,
                                  np.zeros(3))
    assert full[2] == 1000e-15 and early[2] < 200e-15
    g = lambda u: math.sqrt(1 + u @ u)
    assert abs(g(early[1]) / g(full[1]) - 1) < 1e-9
    assert early[3] < full[3]


def test_energy_check_once_per_period(orc):
    """Stop rule: the energy is compared at the first accepted step end at
    least 0.999 optical period after the previous check (the first one after
    birth).  In a uniform magnetic field gamma is constant, so a loose
    tolerance stops the electron at its first check: between 0.999 T and
    0.999 T + h_max after birth."""
    L = orc.laser_intensity(0.8e-6, 3e-6, 30e-15, 1e21, field=orc.UNIFORM_EB,
                            test_B=(0.0, 0.0, 500.0), window=1)
    T = L.lambda_ / C
    A = orc.adaptive(L=L, k_tol=1e-6)
    t0 = -20e-15
    xf, uf, ts, na, nr, st = orc.push_one_adaptive(L, A, t0, 100e-15, np.zeros(3),
                                                   np.array([3.0, 0.0, 1.0]))
    assert st == 0 and 0.999 * T <= ts - t0 <= 0.999 * T + A.h_max * (1 + 1e-12), (ts - t0) / T


def test_step_budget_and_window_edges(orc):
    L = orc.laser_intensity(0.8e-6, 3e-6, 30e-15, 1e21)
    A = orc.adaptive(L=L, max_steps=5)
    xf, uf, ts, na, nr, st = orc.push_one_adaptive(L, A, -15e-15, 100e-15, np.array([1e-6, 0, 0]),
                                                   np.zeros(3))
    assert st == 1 and np.all(np.isnan(uf)) and math.isnan(ts) and na + nr == 5
    # born at the window end: no step, momentum zero
    z0 = np.array([0.0])
    te = 10 * 30e-15
    out = orc.push_adaptive(L, orc.adaptive(L=L), np.array([te, np.inf]), z0, z0, z0, 2)
    assert out[0][0] == 0.0 and out[6][0] == te and out[7][0] == 0
    assert np.isnan(out[0][1]) and np.isnan(out[6][1])


def test_controller_against_closed_form_stages(orc):
    """Uniform field along x, electron from rest: every stage momentum is
    exact (u linear in t), so the stage derivatives of x are the closed form
    c u/gamma at the stage times.  Driving the published step-size rule with
    them gives the accepted / rejected step counts the oracle must report."""
    E0 = 1e10                      # the motion turns relativistic within ~0.2 fs
    L = orc.laser_intensity(0.8e-6, 3e-6, 30e-15, 1e21, field=orc.UNIFORM_EB,
                            test_E=(E0, 0, 0), window=1)
    k = 2 * math.pi / L.lambda_
    a = QE * E0 / (ME * C)
    c_, A_, b5, b4 = orc.dp_tableau()
    for tol in (1e-10, 1e-12):
        A = orc.adaptive(rtol=tol, atol=tol, h_max=1.0, L=L, k_tol=0.0)
        T_end = 600e-15
        xf, uf, ts, na, nr, st = orc.push_one_adaptive(L, A, 0.0, T_end, np.zeros(3), np.zeros(3))
        # the rule: error = max over components of |y5 - y4| / (atol + rtol max(|y_n|, |y_n+1|)),
        # positions as k x; accept if <= 1; h <- h min(5, max(0.2, 0.9 err^-1/5))
        f = lambda t: -C * a * t / math.sqrt(1 + (a * t) ** 2)
        t, x, h, acc, rej = 0.0, 0.0, L.dt, 0, 0
        while t < T_end:
            hs = min(h, 1.0)
            last = hs >= T_end - t
            if last:
                hs = T_end - t
            fs = [f(t + ci * hs) for ci in c_]
            x5 = x + hs * sum(b5[i] * fs[i] for i in range(7))
            ex = abs(hs * sum((b5[i] - b4[i]) * fs[i] for i in range(7))) * k
            err = ex / (tol + tol * k * max(abs(x), abs(x5)))
            if err <= 1:
                t = T_end if last else t + hs
                x = x5
                acc += 1
                if last:
                    break
            else:
                rej += 1
            fac = 5.0 if err == 0 else min(5.0, max(0.2, 0.9 * err ** -0.2))
            h = hs * fac
        assert st == 0 and ts == T_end
        assert (na, nr) == (acc, rej), (tol, na, nr, acc, rej)
        assert abs(xf[0] / x - 1) < 1e-9
        assert acc > 40 and rej > 0
