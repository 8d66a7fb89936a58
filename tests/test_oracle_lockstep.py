"""Pins of the oracle's lock-step batches (the paper's batching, Sec. 2: the
cells of a batch share one integrator, one step size and order, and one WRMS
norm over the batch vector, N = B S in Eq. (3)).

* A batch of one cell is the per-cell integration, bit for bit.
* Linear kinetics in batches against scipy's expm, cell by cell.
* Robertson copies against the published t = 40 values.
* The norm is over the whole batch vector: a cell at rest halves the mean
  square of the error, so the batch takes fewer steps than the active cell
  alone; a stiff cell sets the step count of a batch with a slow one.
* A batch fails as a whole; the driver cuts each mechanism's cells, in index
  order, into consecutive batches, each integrated as if on its own.
"""
import numpy as np
import pytest
from scipy.linalg import expm

from paper_2405_01713_amd import workloads as W
from tests.test_oracle_integration import _golden, _linear_K


def test_batch_of_one_is_the_per_cell_integration(oracle):
    w = W.make_workload("s21_r84_262k", 64)
    args = (w["mechs"], w["y0"], 0.0, w["t_out"], w["rtol"], w["atol"])
    y1, s1 = oracle.integrate(*args, T=w["T"])
    yb, sb = oracle.integrate(*args, T=w["T"], lockstep=1)
    assert np.array_equal(y1, yb) and np.array_equal(s1, sb)


@pytest.mark.parametrize("B", [2, 4, 7])
def test_linear_kinetics_in_batches_against_expm(oracle, B):
    m = W.unimolecular_mechanism(6, 12, 2)
    rng = np.random.default_rng(B)
    y0 = rng.uniform(0.1, 1.0, (B, 6))
    rtol, atol = 1e-6, 1e-10
    y, st = oracle.integrate(m, y0, 0.0, 2.0, rtol, atol, lockstep=B)
    E = expm(_linear_K(m) * 2.0)
    assert np.all(st["status"] == 0) and np.all(st["nst"] == st["nst"][0])
    for c in range(B):
        ref = E @ y0[c]
        assert np.all(np.abs(y[c] - ref) <= 100 * rtol * np.abs(ref) + atol)


def test_robertson_copies(oracle):
    m = W.robertson_mechanism()
    y0 = np.tile([1.0, 0.0, 0.0], (3, 1))
    y, st = oracle.integrate(m, y0, 0.0, 40.0, 1e-6, 1e-10, lockstep=3)
    g = _golden("robertson_t40.json")
    assert np.all(st["status"] == 0)
    for c in range(3):
        assert np.allclose(y[c], g["y"], rtol=g["rel_tol"], atol=0)


def _decay(k):
    """Two species, A -> B with rate constant k (a linear system)."""
    return dict(n_species=2, n_reactions=1, reac=np.array([[0, -1, -1]], dtype=np.int32),
                prod=np.array([[1, -1, -1]], dtype=np.int32), lnA=np.log([k]), EaR=np.zeros(1),
                lnK=None, w=np.ones(2))


def test_norm_runs_over_the_batch_vector(oracle):
    m = _decay(5.0)
    rtol, atol = 1e-6, 1e-10
    ya, sa = oracle.integrate(m, np.array([[1.0, 0.0]]), 0.0, 2.0, rtol, atol)
    # the second cell is at rest (y = 0 is an equilibrium): its error is 0
    yb, sb = oracle.integrate(m, np.array([[1.0, 0.0], [0.0, 0.0]]), 0.0, 2.0, rtol, atol,
                              lockstep=2)
    assert np.all(sb["status"] == 0) and np.all(yb[1] == 0.0)
    assert sb["nst"][0] < sa["nst"][0]
    ref = np.array([np.exp(-10.0), 1.0 - np.exp(-10.0)])
    assert np.all(np.abs(yb[0] - ref) <= 100 * rtol * np.abs(ref) + atol)
    # the order of the cells in the batch does not matter
    yc, sc = oracle.integrate(m, np.array([[0.0, 0.0], [1.0, 0.0]]), 0.0, 2.0, rtol, atol,
                              lockstep=2)
    assert sc["nst"][0] < sa["nst"][0] and np.all(yc[0] == 0.0)
    assert np.all(np.abs(yc[1] - ref) <= 100 * rtol * np.abs(ref) + atol)


def test_stiff_cell_sets_the_steps_of_its_batch(oracle):
    """Cells with different rate scales share one step size: the slow cell
    of a batch takes the fast cell's steps."""
    m = W.unimolecular_mechanism(4, 6, 3)
    y0 = np.array([[0.4, 0.3, 0.2, 0.1], [0.1, 0.2, 0.3, 0.4]])
    ks = np.array([np.full(6, 1.0), np.full(6, 1e-3)])  # cell 1: 1000 times slower
    rtol, atol = 1e-6, 1e-10
    _, s1 = oracle.integrate(m, y0, 0.0, 1.0, rtol, atol, kscale=ks)
    yb, sb = oracle.integrate(m, y0, 0.0, 1.0, rtol, atol, kscale=ks, lockstep=2)
    assert s1["nst"][0] > 3 * s1["nst"][1]
    assert sb["nst"][1] == sb["nst"][0] >= 0.7 * s1["nst"][0]
    for c in range(2):
        mc = dict(m, lnA=m["lnA"] + np.log(ks[c]))
        ref = expm(_linear_K(mc) * 1.0) @ y0[c]
        assert np.all(np.abs(yb[c] - ref) <= 100 * rtol * np.abs(ref) + atol)


def test_batches_fail_as_a_whole(oracle):
    w = W.make_workload("s21_r84_262k", 8)
    y0 = w["y0"].copy()
    y0[2, 5] = np.nan
    y, st = oracle.integrate(w["mechs"], y0, 0.0, w["t_out"], w["rtol"], w["atol"], T=w["T"],
                             lockstep=4)
    assert np.all(st["status"][:4] == -9) and np.all(st["status"][4:] == 0)
    assert np.array_equal(y[[0, 1, 3]], y0[[0, 1, 3]])
    yr, sr = oracle.integrate(w["mechs"], y0[4:], 0.0, w["t_out"], w["rtol"], w["atol"],
                              T=w["T"][4:], lockstep=4)
    assert np.array_equal(y[4:], yr) and np.array_equal(st[4:], sr)
    # too much work ends the whole batch at the same time
    y, st = oracle.integrate(w["mechs"], w["y0"], 0.0, w["t_out"], w["rtol"], w["atol"],
                             T=w["T"], lockstep=4, max_steps=50)
    tr = st["t_reached"].reshape(2, 4)
    assert np.all(st["status"] == -1) and np.all(tr == tr[:, :1])


def test_batches_are_consecutive_cells_of_each_mechanism(oracle):
    w = W.make_workload("mixed_s9_s53_1m", 23)
    B = 3
    y, st = oracle.integrate(w["mechs"], w["y0"], 0.0, w["t_out"], w["rtol"], w["atol"],
                             T=w["T"], cell_mech=w["cell_mech"], lockstep=B)
    assert np.all(st["status"] == 0)
    for mm, mech in enumerate(w["mechs"]):
        cells = np.nonzero(w["cell_mech"] == mm)[0]
        for k in range(0, cells.size, B):
            grp = cells[k:k + B]
            yg, sg = oracle.integrate([mech], w["y0"][grp], 0.0, w["t_out"], w["rtol"],
                                      w["atol"], T=w["T"][grp], lockstep=B)
            assert np.array_equal(y[grp], yg) and np.array_equal(st[grp], sg)
            assert np.all(sg["nst"] == sg["nst"][0])
