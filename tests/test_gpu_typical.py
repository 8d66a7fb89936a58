"""GPU tests of the typical-value absolute tolerances (Sec. 4.1.3, Eq. (9)).

The typical values are extremes and one rounded mean, so the device values
must equal the oracle's bit for bit; integrations that use the resulting
tolerances are checked against the oracle run with the same tolerance
vectors; the splitting loop that recomputes them every other outer step is
captured in a graph and replayed against the eager run.
"""
import numpy as np
import pytest

from paper_2405_01713_amd import workloads as W

pytestmark = pytest.mark.gpu


def _typical_gpu(integ, eta):
    import torch
    typ = torch.full((len(integ.mechs), integ.S_max), -7.0, dtype=torch.float64,
                     device=integ.dev)
    integ.typical_atol(eta, typ)
    torch.cuda.synchronize()
    return typ.cpu().numpy()


def _integrator(w, **opts):
    from paper_2405_01713_amd import bdfx
    return bdfx.Integrator(w["mechs"], w["y0"], w["rtol"], w["atol"], T=w.get("T"),
                           cell_mech=w.get("cell_mech"), **opts)


@pytest.mark.parametrize("n", [1, 2, 5000, 262144])
def test_typical_values_bit_exact_single(oracle, n):
    w = W.make_workload("s21_r84_262k", n)
    y = w["y0"].copy()
    rng = np.random.default_rng(n)
    if n > 2:
        y[:, 3] = -rng.uniform(0, 1e-3, n)   # negative everywhere: default typical value
        y[:, 4] = 0.0                          # absent everywhere
        y[n // 2, 5] = np.nan                  # a NaN entry
    w = dict(w, y0=y)
    integ = _integrator(w, scheduler=1)
    typ = _typical_gpu(integ, 1e-10)
    integ.close()
    to, _ = oracle.typical_atol(y, 1e-10, [21])
    assert np.array_equal(typ, to, equal_nan=True)


@pytest.mark.parametrize("S", [1, 64])
def test_typical_values_species_limits(oracle, S):
    """One species (a pass covers 64 cells; the combine splits the partials
    1,024 ways) and 64 species (one cell per pass; 16 ways), over a cell
    count that fills the block cap and leaves a ragged last pass."""
    if S == 1:
        m = dict(name="sink_s1", n_species=1, n_reactions=1,
                 reac=np.array([[0, -1, -1]], dtype=np.int32),
                 prod=np.full((1, 3), -1, dtype=np.int32), lnA=np.zeros(1), EaR=np.zeros(1),
                 lnK=None, w=np.ones(1))
    else:
        m = W.unimolecular_mechanism(64, 64, 3)
    n = 300007
    rng = np.random.default_rng(S)
    y = rng.uniform(-0.1, 1.0, (n, S))
    y[rng.integers(0, n, 5), rng.integers(0, S, 5)] = rng.uniform(1.0, 2.0, 5)
    integ = _integrator(dict(mechs=[m], y0=y, rtol=1e-6, atol=1e-10), scheduler=1)
    typ = _typical_gpu(integ, 1e-10)
    integ.close()
    to, _ = oracle.typical_atol(y, 1e-10, [S])
    assert np.array_equal(typ, to)


def test_typical_values_bit_exact_mixed(oracle):
    w = W.make_workload("mixed_s9_s53_1m", 3001)
    integ = _integrator(w, scheduler=0)
    typ = _typical_gpu(integ, 1e-8)
    integ.close()
    to, _ = oracle.typical_atol(w["y0"], 1e-8, [9, 53], cell_mech=w["cell_mech"])
    assert np.array_equal(typ, to[:, :53])


def test_mechanism_without_cells_keeps_defaults(oracle):
    w = W.make_workload("mixed_s9_s53_1m", 64)
    cm = np.zeros(64, dtype=np.int32)        # every cell uses mechanism 0
    w = dict(w, cell_mech=cm)
    integ = _integrator(w, scheduler=1)
    typ = _typical_gpu(integ, 1e-10)
    integ.close()
    to, _ = oracle.typical_atol(w["y0"], 1e-10, [9, 53], cell_mech=cm)
    assert np.array_equal(typ, to[:, :53])
    assert np.all(typ[1] == 0.0)


@pytest.mark.parametrize("lu", [64, 32])
def test_integrate_with_typical_atol(oracle, parity, lu):
    w = W.make_workload("s21_r84_262k", 512)
    integ = _integrator(w, scheduler=1, lu_precision=lu)
    integ.typical_atol(1e-10)
    integ.integrate(0.0, w["t_out"])
    y, st = integ.state(), integ.cell_stats()
    # eta = 0: back to the options' atol
    integ.set_state(w["y0"])
    integ.typical_atol(0.0)
    integ.integrate(0.0, w["t_out"])
    y_fixed = integ.state()
    integ.close()
    _, atol = oracle.typical_atol(w["y0"], 1e-10, [21])
    wt = dict(w, atol=atol[0])
    yo, sto = oracle.integrate(w["mechs"], w["y0"], 0.0, w["t_out"], w["rtol"], atol[0], T=w["T"])
    assert np.all(st["status"] == 0) and np.all(sto["status"] == 0)
    parity(y, yo, wt, f"typical atol lu{lu}")
    yf, _ = oracle.integrate(w["mechs"], w["y0"], 0.0, w["t_out"], w["rtol"], w["atol"], T=w["T"])
    parity(y_fixed, yf, w, f"fixed atol after reset lu{lu}")


def _oracle_loop_typical(oracle, w, n_outer, seed, every, eta, rtol, max_steps=5000):
    ms, cm = w["mechs"], w["cell_mech"]
    S = [m["n_species"] for m in ms]
    y, dt = w["y0"].copy(), w["t_out"]
    atol = None
    for k in range(n_outer):
        y = oracle.perturb(y, [S[m] for m in cm], [ms[m]["w"] for m in cm], seed, k, w["perturb"])
        if k % every == 0:
            _, atol = oracle.typical_atol(y, eta, S, cell_mech=cm)
        for m in range(len(ms)):
            sel = cm == m
            ym, st = oracle.integrate(ms[m], y[sel], k * dt, (k + 1) * dt, rtol, atol[m],
                                      T=w["T"][sel],
                                      max_steps=max_steps)
            assert np.all(st["status"] == 0)
            y[sel] = ym
    return y


def test_outer_loop_with_typical_reset_in_graph(oracle):
    """Splitting loop of the mixed batch with the typical values recomputed
    at outer steps 0 and 2: eager vs the oracle's composed loop, graph
    replays vs eager bit for bit."""
    import torch
    w = W.make_workload("mixed_s9_s53_1m", 300)
    n_outer, seed, every, eta = 4, 5, 2, 1e-10
    integ = _integrator(w, scheduler=1)
    y0 = integ.y.clone()
    integ.outer_loop(n_outer, w["t_out"], seed, w["perturb"], typical_every=every, eta=eta)
    torch.cuda.synchronize()
    y_eager, st_eager = integ.state(), integ.cell_stats()
    g = integ.capture_outer_loop(n_outer, w["t_out"], seed, w["perturb"], typical_every=every,
                                 eta=eta)
    for rep in range(3):
        integ.y.copy_(y0)
        integ.typical_atol(0.0)   # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(integ.state(), y_eager), f"replay {rep}"
        assert np.array_equal(integ.cell_stats(), st_eager), f"replay {rep}"
    integ.close()
    assert np.all(st_eager["status"] == 0)
    yo = _oracle_loop_typical(oracle, w, n_outer, seed, every, eta, w["rtol"])
    # per-cell bar with the tolerances in force: 10 rtol |y| + atol_i of the
    # cell's mechanism, for >= 99 % of entries, and 100 x for all
    _, atol = oracle.typical_atol(w["y0"], eta, [9, 53], cell_mech=w["cell_mech"])
    S = np.array([w["mechs"][m]["n_species"] for m in w["cell_mech"]])
    own = np.arange(y_eager.shape[1])[None, :] < S[:, None]
    err = np.abs(y_eager - yo)[own]
    scale = (w["rtol"] * np.abs(yo))[own]
    a_min = min(atol[0][:9].min(), atol[1][:53].min())
    assert np.mean(err <= 10 * scale + a_min) >= 0.99
    assert np.all(err <= 100 * (scale + 1e-10))
