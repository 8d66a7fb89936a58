"""GPU tests of non-isothermal cells (temperature as the last state entry,
rate constants re-evaluated from it, adiabatic constant-volume energy
balance): parity with the oracle in both Newton-matrix precisions, with
forcing, in a batch mixed with an isothermal mechanism, on a tiny system,
schedule independence, the outer loop (the perturbation leaves the
temperature alone), and typical values that include the temperature."""
import numpy as np
import pytest

from paper_2405_01713_amd import workloads as W
from tests.conftest import assert_parity_global

pytestmark = pytest.mark.gpu


def _gpu(w, **opts):
    import torch
    from paper_2405_01713_amd import bdfx
    integ = bdfx.Integrator(w["mechs"], w["y0"], w["rtol"], w["atol"], T=w.get("T"),
                            forcing=w.get("F"), cell_mech=w.get("cell_mech"), **opts)
    integ.integrate(0.0, w["t_out"])
    torch.cuda.synchronize()
    y, st = integ.state(), integ.cell_stats()
    integ.close()
    return y, st


def _energy(m, x):
    S = m["n_species"]
    return np.sum(x[:, :S] * (m["u0"] + m["cv"] * x[:, S:S + 1]), axis=1)


@pytest.mark.parametrize("lu", [64, 32])
def test_thermal_parity(oracle, lu):
    w = W.make_workload("s21_r84_thermal_262k", 512)
    y, st = _gpu(w, scheduler=1, lu_precision=lu)
    yo, sto = oracle.integrate(w["mechs"], w["y0"], 0.0, w["t_out"], w["rtol"], w["atol"])
    assert np.all(st["status"] == 0) and np.all(sto["status"] == 0)
    assert np.median(np.abs(y[:, 21] - w["y0"][:, 21])) > 100.0  # the temperature moves
    assert_parity_global(y, yo, w, oracle, f"thermal lu{lu}")
    m = w["mechs"][0]
    e0 = _energy(m, w["y0"])
    drift_gpu = np.abs(_energy(m, y) - e0) / np.abs(e0)
    drift_orc = np.abs(_energy(m, yo) - e0) / np.abs(e0)
    assert drift_gpu.max() <= 10 * drift_orc.max() + 1e-9


def test_thermal_schedules_identical():
    w = W.make_workload("s21_r84_thermal_262k", 300)
    ys, sts = _gpu(w, scheduler=0)
    yq, stq = _gpu(w, scheduler=1, queue_chunk=3)
    assert np.array_equal(ys, yq) and np.array_equal(sts, stq)


def test_thermal_forcing(oracle):
    w = W.make_workload("s21_r84_thermal_262k", 512)
    rng = np.random.default_rng(31)
    F = rng.uniform(-1.0, 1.0, w["y0"].shape) * 1e2
    F[:, 21] = rng.uniform(-1e6, 1e6, 512)  # heating / cooling rate (K/s)
    w = dict(w, F=F)
    y, st = _gpu(w, scheduler=1)
    yo, sto = oracle.integrate(w["mechs"], w["y0"], 0.0, w["t_out"], w["rtol"], w["atol"], F=F)
    assert np.all(st["status"] == 0) and np.all(sto["status"] == 0)
    assert_parity_global(y, yo, w, oracle, "thermal forcing")


def test_thermal_mixed_with_isothermal(oracle):
    """A 9-species non-isothermal mechanism (10 state entries) next to the
    53-species isothermal one: per-bin state lengths, one batch."""
    m9 = W.thermal_mechanism(W.synthetic_mechanism(9, 30, W.MECH_SEED_S9))
    m53 = W.synthetic_mechanism(53, 325, W.MECH_SEED_S53)
    N = 400
    c = W.mixed_cells([m9, m53], N, 8, (1000.0, 2500.0))
    y0 = c["y0"].copy()
    cm = c["cell_mech"]
    y0[cm == 0, 9] = c["T"][cm == 0]  # temperature entry of the non-isothermal cells
    atol = np.full(53, 1e-10)
    atol[9] = 1e-6
    w = dict(mechs=[m9, m53], y0=y0, T=c["T"], cell_mech=cm, rtol=1e-6, atol=atol, t_out=1e-5)
    from tests.conftest import assert_parity
    ref = {}
    for sched in (0, 1):
        y, st = _gpu(w, scheduler=sched)
        assert np.all(st["status"] == 0)
        for m_, mech in enumerate((m9, m53)):
            sel = cm == m_
            n = 10 if m_ == 0 else 53
            # one atol vector per state index serves both mechanisms
            ws = dict(mechs=[mech], y0=y0[sel, :n], T=c["T"][sel], rtol=1e-6, atol=atol[:n],
                      t_out=1e-5)
            if m_ not in ref:
                ref[m_], sto = oracle.integrate(ws["mechs"], ws["y0"], 0.0, 1e-5, 1e-6, atol[:n],
                                                T=ws["T"])
                assert np.all(sto["status"] == 0)
            check = assert_parity_global if mech.get("cv") is not None else assert_parity
            check(y[sel, :n], ref[m_], ws, oracle, f"mixed sched{sched} mech{m_}")
        # columns past a mechanism's state are untouched
        assert np.all(y[cm == 0, 10:] == y0[cm == 0, 10:])


def test_thermal_tiny_system(oracle):
    m = dict(n_species=3, n_reactions=2,
             reac=np.array([[0, 0, -1], [0, 1, -1]], dtype=np.int32),
             prod=np.array([[1, -1, -1], [2, -1, -1]], dtype=np.int32),
             lnA=np.log([3e3, 5e3]), EaR=np.array([2000.0, 4000.0]), lnK=np.log([4.0, 2.0]),
             w=np.array([1.0, 2.0, 3.0]), cv=np.array([1.5, 2.5, 3.0]),
             u0=np.array([0.0, -800.0, -1500.0]))
    rng = np.random.default_rng(2)
    y0 = np.column_stack([rng.uniform(0.3, 0.7, 64), rng.uniform(0, 0.2, 64),
                          rng.uniform(0, 0.1, 64), rng.uniform(900, 1500, 64)])
    atol = np.array([1e-12] * 3 + [1e-6])
    w = dict(mechs=[m], y0=y0, rtol=1e-8, atol=atol, t_out=2e-3)
    y, st = _gpu(w, scheduler=1)
    yo, sto = oracle.integrate([m], y0, 0.0, 2e-3, 1e-8, atol)
    assert np.all(st["status"] == 0) and np.all(sto["status"] == 0)
    err = np.abs(y - yo)
    assert np.mean(err <= 10 * 1e-8 * np.abs(yo) + atol) >= 0.99
    assert np.all(err <= 100 * (1e-8 * np.abs(yo) + atol))


def test_thermal_outer_loop_and_typical(oracle):
    import torch
    from paper_2405_01713_amd import bdfx
    w = W.make_workload("s21_r84_thermal_262k", 256)
    integ = bdfx.Integrator(w["mechs"], w["y0"], w["rtol"], w["atol"], scheduler=1)
    # the perturbation changes species only
    integ.perturb(7, 0, 0.01)
    torch.cuda.synchronize()
    yp = integ.state()
    assert np.array_equal(yp[:, 21], w["y0"][:, 21])
    m = w["mechs"][0]
    ypo = oracle.perturb(w["y0"], [21] * 256, [m["w"]] * 256, 7, 0, 0.01)
    assert np.array_equal(yp, ypo)
    # typical values cover the 22 state entries, the temperature included
    typ = torch.zeros((1, 22), dtype=torch.float64, device=integ.dev)
    integ.typical_atol(1e-10, typ)
    torch.cuda.synchronize()
    to, _ = oracle.typical_atol(yp, 1e-10, [22])
    assert np.array_equal(typ.cpu().numpy(), to)
    integ.close()
