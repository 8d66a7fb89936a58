"""Pins of the oracle's typical-value absolute tolerances (Sec. 4.1.3, Eq. (9)).

The typical value of a species is half the sum of its smallest and largest
value over the domain; atol_i = eta times it, with the paper's default of 1
where no positive typical value exists.  Pinned by hand-computed values, by
brute force over tiny inputs, by the per-mechanism split of a mixed batch and
by invariance under reordering the cells.
"""
import numpy as np


def test_hand_values(oracle):
    y = np.array([[1.0, 2.0, -1.0, 0.0],
                  [3.0, 0.5, -2.0, 0.0],
                  [2.0, 4.0, -3.0, 0.0]])
    typ, atol = oracle.typical_atol(y, 1e-10, [4])
    assert np.array_equal(typ[0], [2.0, 2.25, -2.0, 0.0])
    # species 2 (all negative) and 3 (all zero) fall back to a typical value of 1
    assert np.array_equal(atol[0], [2.0e-10, 2.25e-10, 1.0e-10, 1.0e-10])


def test_brute_force_tiny(oracle):
    rng = np.random.default_rng(5)
    for trial in range(20):
        N, S = int(rng.integers(1, 7)), int(rng.integers(1, 5))
        y = rng.uniform(-0.2, 1.0, (N, S + 2))
        eta = 10.0 ** rng.uniform(-14, -6)
        typ, atol = oracle.typical_atol(y, eta, [S])
        for i in range(S):
            lo = hi = y[0, i]
            for c in range(1, N):
                lo = min(lo, y[c, i])
                hi = max(hi, y[c, i])
            t = (lo + hi) / 2
            assert typ[0, i] == t
            assert atol[0, i] == (t if t > 0 else 1.0) * eta
            assert lo <= typ[0, i] <= hi
        # columns beyond the species count are not tolerances of this mechanism
        assert np.all(typ[0, S:] == 0.0) and np.all(atol[0, S:] == eta)


def test_mixed_mechanisms_are_separate(oracle):
    rng = np.random.default_rng(7)
    N, ldy = 40, 6
    y = rng.uniform(0.0, 1.0, (N, ldy))
    cm = rng.integers(0, 3, N)
    cm[:3] = [0, 1, 2]
    S = [6, 2, 4]
    typ, atol = oracle.typical_atol(y, 1e-8, S, cell_mech=cm)
    for m in range(3):
        t1, a1 = oracle.typical_atol(y[cm == m], 1e-8, [S[m]])
        assert np.array_equal(typ[m], t1[0]) and np.array_equal(atol[m], a1[0])
    # a mechanism without cells keeps the default
    typ2, atol2 = oracle.typical_atol(y, 1e-8, [6, 2, 4, 5], cell_mech=cm)
    assert np.all(typ2[3] == 0.0) and np.all(atol2[3] == 1e-8)


def test_order_of_cells_does_not_matter(oracle):
    rng = np.random.default_rng(9)
    y = rng.lognormal(-5, 3, (500, 21))
    typ, atol = oracle.typical_atol(y, 1e-10, [21])
    perm = rng.permutation(500)
    typ_p, atol_p = oracle.typical_atol(y[perm], 1e-10, [21])
    assert np.array_equal(typ, typ_p) and np.array_equal(atol, atol_p)
