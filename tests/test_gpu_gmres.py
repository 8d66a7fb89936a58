"""GPU tests of the inexact Newton iteration with matrix-free GMRES (Table 1,
approaches 1A/1B): parity with the oracle run with the same Krylov dimension
(21 and 53 species, non-isothermal cells, Robertson, typical-value
tolerances), schedule independence, the statistics, and the option checks."""
import numpy as np
import pytest

from paper_2405_01713_amd import workloads as W
from tests.conftest import assert_parity_global

pytestmark = pytest.mark.gpu


def _gpu(w, maxl, **opts):
    import torch
    from paper_2405_01713_amd import bdfx
    integ = bdfx.Integrator(w["mechs"], w["y0"], w["rtol"], w["atol"], T=w.get("T"),
                            kscale=w.get("kscale"), cell_mech=w.get("cell_mech"),
                            gmres_maxl=maxl, **opts)
    integ.integrate(0.0, w["t_out"])
    torch.cuda.synchronize()
    y, st, summ = integ.state(), integ.cell_stats(), integ.summary()
    integ.close()
    return y, st, summ


def _oracle(oracle, w, maxl):
    return oracle.integrate(w["mechs"], w["y0"], 0.0, w["t_out"], w["rtol"], w["atol"],
                            T=w.get("T"), kscale=w.get("kscale"), cell_mech=w.get("cell_mech"),
                            gmres_maxl=maxl)


def test_gmres_parity_21_species(oracle, parity):
    w = dict(W.make_workload("s21_r84_262k", 512), t_out=1e-8)
    y, st, summ = _gpu(w, 10, scheduler=1)
    yo, sto = _oracle(oracle, w, 10)
    assert np.all(st["status"] == 0) and np.all(sto["status"] == 0)
    parity(y, yo, w, "gmres maxl 10")
    assert np.all(st["nsetups"] == 0) and np.all(st["nli"] > 0)
    # the same work as the oracle's, and one right-hand side per iteration
    assert abs(st["nli"].mean() / sto["nli"].mean() - 1.0) < 0.03
    assert abs(st["nst"].mean() / sto["nst"].mean() - 1.0) < 0.03
    assert np.all(st["nfe"] - st["nli"] >= st["nni"] + 1)
    assert summ["nli"] == int(st["nli"].sum()) and summ["ncfl"] == int(st["ncfl"].sum())
    assert summ["nsetups"] == 0


def test_gmres_short_krylov_space(oracle):
    """5 Krylov vectors: unconverged solves accepted on first Newton
    iterations make the result sensitive to round-off (global bar)."""
    w = dict(W.make_workload("s21_r84_262k", 512), t_out=1e-8)
    y, st, _ = _gpu(w, 5, scheduler=1)
    yo, sto = _oracle(oracle, w, 5)
    assert np.all(st["status"] == 0) and np.all(sto["status"] == 0)
    assert st["ncfl"].sum() > 0
    assert_parity_global(y, yo, w, oracle, "gmres maxl 5", min_frac=0.5)


def test_gmres_schedules_identical():
    w = dict(W.make_workload("s21_r84_262k", 300), t_out=1e-8)
    ys, sts, _ = _gpu(w, 10, scheduler=0)
    yq, stq, _ = _gpu(w, 10, scheduler=1, queue_chunk=3)
    assert np.array_equal(ys, yq) and np.array_equal(sts, stq)


def test_gmres_53_species(oracle):
    w = dict(W.make_workload("s53_r325_262k_fp32lu", 128), t_out=1e-8)
    y, st, _ = _gpu(w, 10, scheduler=1)
    yo, sto = _oracle(oracle, w, 10)
    assert np.all(st["status"] == 0) and np.all(sto["status"] == 0)
    assert np.all(st["nsetups"] == 0)
    assert_parity_global(y, yo, w, oracle, "gmres 53 species")


def test_gmres_non_isothermal(oracle):
    w = dict(W.make_workload("s21_r84_thermal_262k", 256), t_out=1e-8)
    y, st, _ = _gpu(w, 10, scheduler=1)
    yo, sto = _oracle(oracle, w, 10)
    assert np.all(st["status"] == 0) and np.all(sto["status"] == 0)
    assert_parity_global(y, yo, w, oracle, "gmres non-isothermal")


def test_gmres_robertson(oracle, parity):
    w = W.make_workload("robertson_4k", 256)
    y, st, _ = _gpu(w, 5, scheduler=1)
    yo, sto = _oracle(oracle, w, 5)
    assert np.all(st["status"] == 0) and np.all(sto["status"] == 0)
    parity(y, yo, w, "gmres robertson")


def test_gmres_typical_tolerances(oracle, parity):
    """Approach 1B: per-species tolerances from typical values."""
    w = dict(W.make_workload("s21_r84_262k", 256), t_out=1e-8)
    _, atol = oracle.typical_atol(w["y0"], 1e-10, [21])
    w = dict(w, atol=atol[0])
    y, st, _ = _gpu(w, 10, scheduler=1)
    yo, sto = _oracle(oracle, w, 10)
    assert np.all(st["status"] == 0) and np.all(sto["status"] == 0)
    parity(y, yo, w, "gmres typical values")


def test_gmres_option_checks():
    from paper_2405_01713_amd import bdfx
    w = W.make_workload("s21_r84_262k", 8)
    for bad in (dict(gmres_maxl=11), dict(gmres_maxl=-1),
                dict(gmres_maxl=5, jacobian=bdfx.BDFX_JAC_DQ),
                dict(gmres_maxl=5, record_steps=100)):
        with pytest.raises(bdfx.BdfxError):
            bdfx.Integrator(w["mechs"], w["y0"], w["rtol"], w["atol"], T=w["T"], **bad)
    # two cells per wave falls back to one for GMRES; the FP32 option has no matrix to act on
    import torch
    integ = bdfx.Integrator(w["mechs"], w["y0"], w["rtol"], w["atol"], T=w["T"], gmres_maxl=5,
                            cells_per_wave=2, lu_precision=32, scheduler=1)
    integ.integrate(0.0, 1e-8)
    torch.cuda.synchronize()
    assert np.all(integ.cell_stats()["status"] == 0)
    assert all(t["cells_per_wave"] == 1 for t in integ.tuning())
    integ.close()


def test_gmres_forcing(oracle, parity):
    import torch
    from paper_2405_01713_amd import bdfx
    w = dict(W.make_workload("s21_r84_262k", 128), t_out=1e-8)
    rng = np.random.default_rng(21)
    F = rng.uniform(-1.0, 1.0, w["y0"].shape) * 1e2
    w = dict(w, F=F)
    integ = bdfx.Integrator(w["mechs"], w["y0"], w["rtol"], w["atol"], T=w["T"], forcing=F,
                            scheduler=1, gmres_maxl=10)
    integ.integrate(0.0, w["t_out"])
    torch.cuda.synchronize()
    y, st = integ.state(), integ.cell_stats()
    integ.close()
    yo, sto = oracle.integrate(w["mechs"], w["y0"], 0.0, w["t_out"], w["rtol"], w["atol"],
                               T=w["T"], F=F, gmres_maxl=10)
    assert np.all(st["status"] == 0) and np.all(sto["status"] == 0)
    parity(y, yo, w, "gmres forcing")


def test_gmres_graph_replay():
    """GMRES in the captured outer loop: replays equal the eager run bit for bit."""
    import torch
    from paper_2405_01713_amd import bdfx
    w = W.make_workload("s21_r84_262k", 120)
    integ = bdfx.Integrator(w["mechs"], w["y0"], w["rtol"], w["atol"], T=w["T"], scheduler=1,
                            gmres_maxl=10)
    y0 = integ.y.clone()
    integ.outer_loop(2, 1e-8, 9, 0.01)
    torch.cuda.synchronize()
    y_eager, st_eager = integ.state(), integ.cell_stats()
    assert np.all(st_eager["status"] == 0)
    g = integ.capture_outer_loop(2, 1e-8, 9, 0.01)
    for rep in range(3):
        integ.y.copy_(y0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(integ.state(), y_eager), f"replay {rep}"
        assert np.array_equal(integ.cell_stats(), st_eager), f"replay {rep}"
    integ.close()


def test_gmres_largest_size_all_lanes(oracle):
    """64 species, 10 Krylov vectors: every lane holds a species, and the
    Krylov area is at its largest."""
    m = W.synthetic_mechanism(64, 150, 5)
    c = W.cell_states(m, 64, seed=8)
    w = dict(mechs=[m], y0=c["y0"], T=c["T"], rtol=1e-6, atol=1e-10, t_out=1e-8)
    y, st, _ = _gpu(w, 10, scheduler=1)
    yo, sto = _oracle(oracle, w, 10)
    assert np.all(st["status"] == 0) and np.all(sto["status"] == 0)
    assert_parity_global(y, yo, w, oracle, "gmres S=64")
