"""Pins of the oracle's error estimates and initial step against the mathematics.

The step controller rests on three estimates the paper leaves to the reader
(Sec. 2 states only that the local error is tested in the WRMS norm of Eq. (3)
and that step size and order are then re-chosen):

* the local-error estimate Cerr * e of an accepted step, Cerr = 1/(l_1 xi_{q+1});
* the order-selection estimates of the neighbouring orders q - 1 and q + 1;
* the initial step size.

None of the checks below compares the oracle with itself.  The truth is the
exact solution: scipy's expm for linear kinetics, the Riccati closed form of
A + B <=> C, the exact Nordsieck arrays of those solutions, and the local error
actually committed by a BDF step started from exact past values.  Every ratio
"measured / estimated" must tend to 1 as h -> 0, its distance from 1 shrinking
like h.  The ``check_*`` functions are also run against copies of the oracle
with planted mistakes (tests/test_oracle_pins_bite.py), where they must fail.
"""
import math

import numpy as np
from scipy.linalg import expm

# --------------------------------------------------------------------------
# test problems with exact solutions
# --------------------------------------------------------------------------


def chain_mechanism(k1=3.0, k2=5.0):
    """A -> B -> C, first order: y' = K y with eigenvalues 0, -k1, -k2."""
    return dict(n_species=3, n_reactions=2,
                reac=np.array([[0, -1, -1], [1, -1, -1]], dtype=np.int32),
                prod=np.array([[1, -1, -1], [2, -1, -1]], dtype=np.int32),
                lnA=np.log([k1, k2]), EaR=np.zeros(2), lnK=None)


def chain_K(k1=3.0, k2=5.0):
    return np.array([[-k1, 0.0, 0.0], [k1, -k2, 0.0], [0.0, k2, 0.0]])


class Linear:
    """y(t) = expm(K t) y0 and its derivatives K^j y(t)."""

    def __init__(self, K, y0):
        self.K, self.y0 = K, np.asarray(y0, dtype=float)

    def y(self, t):
        return expm(self.K * t) @ self.y0

    def deriv(self, t, j):
        return np.linalg.matrix_power(self.K, j) @ self.y(t)

    def flow(self, h, y):
        """Exact solution after h from state y (the local solution)."""
        return expm(self.K * h) @ y


class Riccati:
    """A + B <=> C with k_f, k_r: A' = -kf A (A - d) + kr (s - A), d = A - B and
    s = A + C conserved; (A - r1)/(A - r2) decays as exp(-kf (r1 - r2) t)."""

    def __init__(self, kf, Kc, y0):
        self.kf, self.kr = kf, kf / Kc
        A0, B0, C0 = y0
        self.d, self.s = A0 - B0, A0 + C0
        a, b, c = -kf, kf * self.d - self.kr, self.kr * self.s
        disc = math.sqrt(b * b - 4 * a * c)
        r = sorted(((-b - disc) / (2 * a), (-b + disc) / (2 * a)))
        self.r2, self.r1 = r
        self.Q0 = (A0 - self.r1) / (A0 - self.r2)
        self.mech = dict(n_species=3, n_reactions=1,
                         reac=np.array([[0, 1, -1]], dtype=np.int32),
                         prod=np.array([[2, -1, -1]], dtype=np.int32),
                         lnA=np.array([math.log(kf)]), EaR=np.zeros(1),
                         lnK=np.array([math.log(Kc)]))

    def y(self, t):
        Q = self.Q0 * math.exp(-self.kf * (self.r1 - self.r2) * t)
        A = (self.r1 - self.r2 * Q) / (1 - Q)
        return np.array([A, A - self.d, self.s - A])


def interpolant_nordsieck(sol, t_last, past_sizes, q, h):
    """Nordsieck array, in units of h, at t_last of the degree-q polynomial
    through the exact values at t_last and the q earlier points
    t_last - past_sizes[0], t_last - past_sizes[0] - past_sizes[1], ..."""
    nodes = [t_last]
    for k in range(q):
        nodes.append(nodes[-1] - past_sizes[k])
    x = (np.array(nodes) - t_last) / h
    V = np.vander(x, q + 1, increasing=True)
    Y = np.array([sol.y(t) for t in nodes])
    return np.linalg.solve(V, Y)  # row j = coefficient of x^j


def step_from_exact_history(O, sol, mech, q, h, t_last, past_sizes):
    """One order-q step of size h from the interpolant of exact past values.
    Returns (local error d = y(t_n) - y_n, predictor error y(t_n) - P(t_n), e, Cerr)."""
    kf, kr = O.rates(mech)
    z = interpolant_nordsieck(sol, t_last, past_sizes, q, h)
    yo, eo, co, _ = O.steps(mech, kf, kr, z, q, [h], past_sizes)
    yt = sol.y(t_last + h)
    return yt - yo[0], yt - z.sum(axis=0), eo[0], co[0]


CONSTANT = [1.0] * 6
RAGGED = [1.6, 0.7, 1.3, 0.55, 1.9, 1.0]  # past step sizes in units of h


def _dev(measured, estimate):
    """Relative distance of two error vectors, ||measured - estimate|| / ||estimate||
    (a vector comparison: a component whose leading term happens to vanish
    carries no weight)."""
    return float(np.linalg.norm(measured - estimate) / np.linalg.norm(estimate))


# --------------------------------------------------------------------------
# local-error estimate of an accepted step
# --------------------------------------------------------------------------


def check_local_error_constant_from_exact_history(O):
    """Started from exact past values, the corrector's local error is -Cerr
    times the predictor's error, to leading order, for any step history:
    ||d + Cerr (y(t_n) - P(t_n))|| / ||Cerr (y(t_n) - P(t_n))|| -> 0, falling
    like h (halving h halves it).  Run at constant and at ragged step-size
    ratios, q = 1..5, on linear kinetics and on the nonlinear A + B <=> C."""
    lin = Linear(chain_K(), [1.0, 0.3, 0.2])
    ric = Riccati(20.0, 50.0, [0.3, 0.2, 0.05])
    for sol, mech, h0, t_last in ((lin, chain_mechanism(), 0.02, 0.4),
                                  (ric, ric.mech, 0.02, 0.3)):
        for q in range(1, 6):
            for pattern in (CONSTANT, RAGGED):
                devs = []
                for h in (h0, h0 / 2, h0 / 4):
                    d, Ep, e, Cerr = step_from_exact_history(
                        O, sol, mech, q, h, t_last, [p * h for p in pattern])
                    devs.append(_dev(d, -Cerr * Ep))
                _first_order(devs, 0.35, (q, pattern))


def _first_order(devs, bound, label):
    """Distances at h, h/2, h/4 that fall like h towards 0."""
    assert devs[0] < bound, (label, devs)
    for a, b in zip(devs, devs[1:]):
        assert 0.4 < b / a < 0.6, (label, devs)


def _taylor_start(lin, h, q):
    return np.array([h ** j * lin.deriv(0.0, j) / math.factorial(j) for j in range(q + 1)])


def _running(O, lin, mech, q, hseq):
    kf, kr = O.rates(mech)
    z = _taylor_start(lin, hseq[0], q)
    return O.steps(mech, kf, kr, z, q, hseq, [hseq[0]] * 6)


def check_local_error_estimate_in_a_running_integration(O):
    """In a running fixed-order integration the estimate Cerr e of a step is
    its local error: at the last step of a run over [0, 1.2], the local error
    of a step of the same size from exact values at the run's own past nodes
    approaches -Cerr e (relative distance falling like h).  Constant steps,
    and steps whose size varies smoothly along the solution, so that the
    ratios xi change from step to step.  (The per-step growth of the global
    error is a different quantity, l_1 Cerr e at constant steps.)"""
    lin = Linear(chain_K(), [1.0, 0.3, 0.2])
    mech = chain_mechanism()
    for q in range(1, 6):
        for smooth in (False, True):
            devs = []
            for h in (0.02, 0.01, 0.005):
                n = int(round(1.2 / h))
                if smooth:
                    hs, t = [], 0.0
                    for _ in range(n):
                        hs.append(h * (1.0 + 0.3 * math.sin(2 * math.pi * t / 0.6)))
                        t += hs[-1]
                else:
                    hs = [h] * n
                yo, eo, co, _ = _running(O, lin, mech, q, hs)
                k = n - 1
                d, _, _, Cerr = step_from_exact_history(
                    O, lin, mech, q, hs[k], float(np.sum(hs[:k])), hs[k - 1::-1][:6])
                assert Cerr == co[k]
                devs.append(_dev(d, -co[k] * eo[k]))
            _first_order(devs, 0.35, (q, smooth))


def test_local_error_constant_from_exact_history(oracle):
    check_local_error_constant_from_exact_history(oracle)


def test_local_error_estimate_in_a_running_integration(oracle):
    check_local_error_estimate_in_a_running_integration(oracle)


# --------------------------------------------------------------------------
# order-selection estimates
# --------------------------------------------------------------------------


def check_lower_order_estimate(O):
    """The order q-1 estimate, computed from the top column of the order-q
    Nordsieck array, equals the local error that an order-(q-1) step of the
    same size actually commits from exact past values (constant steps)."""
    lin = Linear(chain_K(), [1.0, 0.3, 0.2])
    mech = chain_mechanism()
    ones = np.ones(3)
    for q in range(2, 6):
        devs = []
        for h in (0.02, 0.01, 0.005):
            t_last = 0.4
            zq = interpolant_nordsieck(lin, t_last, [h] * 6, q, h)[q]
            est = O.lte_lower(q, zq, ones)
            d, _, _, _ = step_from_exact_history(O, lin, mech, q - 1, h, t_last, [h] * 6)
            devs.append(abs(np.sqrt(np.mean(d ** 2)) / est - 1.0))
        _first_order(devs, 0.3, q)


def check_higher_order_estimate(O):
    """The order q+1 estimate, computed from the corrections of the last two
    steps of a running order-q integration (constant steps), equals the local
    error that an order-(q+1) step of the same size commits from exact past
    values at the same place."""
    lin = Linear(chain_K(), [1.0, 0.3, 0.2])
    mech = chain_mechanism()
    ones = np.ones(3)
    for q in range(1, 5):
        devs = []
        for h in (0.02, 0.01, 0.005):
            n = int(round(0.8 / h))
            yo, eo, co, _ = _running(O, lin, mech, q, [h] * n)
            est = O.lte_higher(q, eo[n - 1], eo[n - 2], h, h, ones)
            t_last = (n - 1) * h  # the last step ends at n h
            d, _, _, _ = step_from_exact_history(O, lin, mech, q + 1, h, t_last, [h] * 6)
            devs.append(abs(np.sqrt(np.mean(d ** 2)) / est - 1.0))
        _first_order(devs, 0.3, q)


def test_lower_order_estimate(oracle):
    check_lower_order_estimate(oracle)


def test_higher_order_estimate(oracle):
    check_higher_order_estimate(oracle)


def test_higher_order_estimate_scales_by_the_step_ratio(oracle):
    """A step-size change between the two corrections is removed by the
    factor (h/h_prev)^(q+1): corrections that are exactly the same polynomial
    error scaled to their own step sizes give a zero estimate."""
    rng = np.random.default_rng(5)
    c = rng.normal(size=6)
    w = np.abs(rng.normal(size=6)) + 0.5
    for q in range(1, 5):
        for ratio in (0.5, 1.7, 3.0):
            hprev, h = 1e-3, 1e-3 * ratio
            eprev = c * hprev ** (q + 1)
            e = c * h ** (q + 1)
            assert oracle.lte_higher(q, e, eprev, h, hprev, w) <= 1e-15 * np.abs(e).max() * w.max()


# --------------------------------------------------------------------------
# initial step
# --------------------------------------------------------------------------


def decay_mechanism(k):
    """A -> B at rate k."""
    return dict(n_species=2, n_reactions=1,
                reac=np.array([[0, -1, -1]], dtype=np.int32),
                prod=np.array([[1, -1, -1]], dtype=np.int32),
                lnA=np.array([math.log(k)]), EaR=np.zeros(1), lnK=None)


def check_initial_step(O):
    """Initial step on linear kinetics, where y'' = K f0 exactly.

    (a) Closed form: with weights w of Eq. (3) at y0, the step is half the
        size whose second-order Taylor term has unit WRMS norm,
        h0 = 0.5 sqrt(2 / ||K f0||_wrms), when that lies inside the bounds.
    (b) Its purpose: the first (order 1) step of the integrator then commits a
        local error of a quarter of the tolerance, ||y_1 - expm(K h0) y0||_wrms
        = h0^2/2 ||y''|| = 1/4, measured on the integrator's own first step.
    (c) Bounds: a short interval caps h0 at 0.1 |t_out - t0|; a vanishing
        second derivative (pure forcing) gives the upper bound
        min(0.1 |t_out - t0|, 1 / max_i |f0_i| / (0.1 |y0_i| + atol)); a large
        |t0| raises h0 to 100 u |t0|.
    """
    rtol, atol = 1e-6, 1e-10
    for k in (1.0, 40.0, 2.5e3):
        m = decay_mechanism(k)
        K = np.array([[-k, 0.0], [k, 0.0]])
        y0 = np.array([1.0, 0.5])
        w = 1.0 / (rtol * np.abs(y0) + atol)
        f0 = K @ y0
        ydd = K @ f0
        h_closed = 0.5 * math.sqrt(2.0 / math.sqrt(np.mean((w * ydd) ** 2)))
        t_out = 1.0
        hub = min(0.1 * t_out, 1.0 / np.max(np.abs(f0) / (0.1 * np.abs(y0) + atol)))
        assert 100 * 2.2e-16 < h_closed < hub
        h0, nfe = O.initial_step(m, y0, 0.0, t_out, rtol, atol)
        assert abs(h0 / h_closed - 1.0) < 1e-8, (k, h0, h_closed)
        assert 2 <= nfe <= 5
        # (b) the integrator's first step
        y1, st = O.integrate(m, y0[None, :], 0.0, t_out, rtol, atol, max_steps=1)
        assert st["nst"][0] == 1 and st["netf"][0] == 0 and st["ncfn"][0] == 0
        assert st["t_reached"][0] == h0
        err = math.sqrt(np.mean((w * (y1[0] - expm(K * h0) @ y0)) ** 2))
        assert abs(err - 0.25) < 0.01, (k, err)
        # (c) short interval
        h0s, _ = O.initial_step(m, y0, 0.0, 1e-2 * h_closed, rtol, atol)
        assert h0s == 0.1 * 1e-2 * h_closed
        # (c) large |t0|: the lower bound 100 u |t| exceeds the estimate
        u = 2.220446049250313e-16
        t0 = 2.0 * h_closed / (100 * u)
        t1 = t0 + 1.0
        h0l, _ = O.initial_step(m, y0, t0, t1, rtol, atol)
        assert h0l == 100 * u * abs(t1)
    # (c) pure forcing: y'' = 0
    m = dict(decay_mechanism(1.0), lnA=np.array([-1000.0]))  # k = 0 exactly
    F = np.array([2.0, -0.5])
    y0 = np.array([1.0, 0.5])
    h0, _ = O.initial_step(m, y0, 0.0, 10.0, rtol, atol, F=F)
    assert h0 == 1.0 / np.max(np.abs(F) / (0.1 * np.abs(y0) + atol))
    h0, _ = O.initial_step(m, y0, 0.0, 0.2, rtol, atol, F=F)
    assert h0 == 0.1 * 0.2


def check_initial_step_nonlinear(O):
    """On the nonlinear A + B <=> C the refinement reaches its fixed point:
    h0 = 0.5 sqrt(2 / ||(f(y0 + h f0) - f0) / h||) evaluated at h = 2 h0 holds
    to within the factor-2 acceptance of the refinement, and the first step's
    local error (against the closed form) is within a factor 2 of 1/4."""
    ric = Riccati(2.0e3, 50.0, [0.3, 0.2, 0.05])
    rtol, atol = 1e-6, 1e-12
    y0 = ric.y(0.0)
    h0, _ = O.initial_step(ric.mech, y0, 0.0, 1e-2, rtol, atol)
    kf, kr = O.rates(ric.mech)
    f0 = O.rhs(ric.mech, kf, kr, y0)
    w = 1.0 / (rtol * np.abs(y0) + atol)
    hh = 2.0 * h0
    ydd = (O.rhs(ric.mech, kf, kr, y0 + hh * f0) - f0) / hh
    h_fix = 0.5 * math.sqrt(2.0 / math.sqrt(np.mean((w * ydd) ** 2)))
    assert 0.5 <= h0 / h_fix <= 2.0
    y1, st = O.integrate(ric.mech, y0[None, :], 0.0, 1e-2, rtol, atol, max_steps=1)
    assert st["t_reached"][0] == h0 and st["netf"][0] == 0
    err = math.sqrt(np.mean((w * (y1[0] - ric.y(h0))) ** 2))
    assert 0.125 <= err <= 0.5, err


def test_initial_step(oracle):
    check_initial_step(oracle)


def test_initial_step_nonlinear(oracle):
    check_initial_step_nonlinear(oracle)
