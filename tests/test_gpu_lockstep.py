"""GPU tests of lock-step batches (the paper's batching, Sec. 2: one step size
and one WRMS norm per batch of cells): parity with the oracle's lock-step
batches, a batch of one equal to per-cell control, ragged batches of a mixed
workload, whole-batch failure, and the option checks."""
import numpy as np
import pytest

from paper_2405_01713_amd import workloads as W

pytestmark = pytest.mark.gpu


def _gpu(w, **opts):
    import torch
    from paper_2405_01713_amd import bdfx
    integ = bdfx.Integrator(w["mechs"], w["y0"], w["rtol"], w["atol"], T=w.get("T"),
                            kscale=w.get("kscale"), cell_mech=w.get("cell_mech"), **opts)
    integ.integrate(0.0, w["t_out"])
    torch.cuda.synchronize()
    y, st = integ.state(), integ.cell_stats()
    integ.close()
    return y, st


def _oracle(oracle, w, B, y0=None):
    return oracle.integrate(w["mechs"], w["y0"] if y0 is None else y0, 0.0, w["t_out"], w["rtol"],
                            w["atol"], T=w.get("T"), kscale=w.get("kscale"),
                            cell_mech=w.get("cell_mech"), lockstep=B)


@pytest.mark.parametrize("B,sched,lu", [(4, 1, 32), (8, 0, 64), (5, 1, 64)])
def test_lockstep_parity(oracle, parity, B, sched, lu):
    w = W.make_workload("s21_r84_262k", 257)  # 257 cells: the last batch is short
    y, st = _gpu(w, lockstep=B, scheduler=sched, lu_precision=lu)
    yo, sto = _oracle(oracle, w, B)
    assert np.all(st["status"] == 0) and np.all(sto["status"] == 0)
    parity(y, yo, w, f"lock-step B{B}")
    # every cell of a batch reports the batch's counters
    nst = st["nst"][:256].reshape(-1, B) if 256 % B == 0 else None
    if nst is not None:
        assert np.all(nst == nst[:, :1])
    # mean step counts move with round-off: the oracle against itself with
    # inputs perturbed by 1e-15 moves them by up to 3.3 % on these batches
    assert abs(st["nst"].mean() / sto["nst"].mean() - 1.0) < 0.06


def test_batch_of_one_is_per_cell_control():
    w = W.make_workload("s21_r84_262k", 200)
    y1, s1 = _gpu(w, scheduler=1, lu_precision=32)
    yb, sb = _gpu(w, lockstep=1, scheduler=1, lu_precision=32)
    rel = np.abs(yb - y1) / (1e-6 * np.abs(y1) + 1e-10)
    assert np.all(sb["status"] == 0)
    assert np.mean(rel <= 10) >= 0.99 and abs(sb["nst"].mean() / s1["nst"].mean() - 1) < 0.01


def test_lockstep_mixed_ragged(oracle, parity):
    w = W.make_workload("mixed_s9_s53_1m", 101)
    y, st = _gpu(w, lockstep=3, scheduler=1, lu_precision=32)
    yo, sto = _oracle(oracle, w, 3)
    assert np.all(st["status"] == 0) and np.all(sto["status"] == 0)
    parity(y, yo, w, "lock-step mixed")
    for mm in range(2):
        cells = np.nonzero(w["cell_mech"] == mm)[0]
        nst = st["nst"][cells]
        for k in range(0, cells.size, 3):
            assert np.all(nst[k:k + 3] == nst[k])


def test_lockstep_batch_fails_as_a_whole(oracle):
    w = W.make_workload("s21_r84_262k", 16)
    y0 = w["y0"].copy()
    y0[5, 3] = np.nan
    w = dict(w, y0=y0)
    y, st = _gpu(w, lockstep=4, scheduler=0)
    yo, sto = _oracle(oracle, w, 4)
    assert np.array_equal(st["status"], sto["status"])
    assert np.all(st["status"][4:8] == -9) and np.all(st["status"][:4] == 0)
    assert np.array_equal(y[[4, 6, 7]], y0[[4, 6, 7]])


def test_lockstep_option_checks():
    from paper_2405_01713_amd import bdfx
    w = W.make_workload("s21_r84_262k", 8)
    for bad in (dict(lockstep=17), dict(lockstep=-1), dict(lockstep=4, gmres_maxl=5),
                dict(lockstep=4, jacobian=bdfx.BDFX_JAC_DQ), dict(lockstep=4, record_steps=10)):
        with pytest.raises(bdfx.BdfxError):
            bdfx.Integrator(w["mechs"], w["y0"], w["rtol"], w["atol"], T=w["T"], **bad)
    wt = W.make_workload("s21_r84_thermal_262k", 8)
    with pytest.raises(bdfx.BdfxError):
        bdfx.Integrator(wt["mechs"], wt["y0"], wt["rtol"], wt["atol"], lockstep=2)
    # 53 species with the FP64 inverse: four waves' LDS exceed 64 KiB
    w53 = W.make_workload("s53_r325_262k_fp32lu", 8)
    with pytest.raises(bdfx.BdfxError):
        bdfx.Integrator(w53["mechs"], w53["y0"], w53["rtol"], w53["atol"], T=w53["T"],
                        lockstep=4, lu_precision=64)


def test_lockstep_graph_replay():
    """The outer loop (perturb, integrate) in lock-step batches: HIP-graph
    replays equal the eager run bit for bit."""
    import torch
    from paper_2405_01713_amd import bdfx
    w = W.make_workload("mixed_s9_s53_1m", 150)
    integ = bdfx.Integrator(w["mechs"], w["y0"], w["rtol"], w["atol"], T=w["T"],
                            cell_mech=w["cell_mech"], scheduler=1, lu_precision=32, lockstep=3)
    y0 = integ.y.clone()
    integ.outer_loop(2, w["t_out"], 5, w["perturb"])
    torch.cuda.synchronize()
    y_eager, st_eager = integ.state(), integ.cell_stats()
    assert np.all(st_eager["status"] == 0)
    g = integ.capture_outer_loop(2, w["t_out"], 5, w["perturb"])
    for rep in range(3):
        integ.y.copy_(y0)
        integ.status.fill_(7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(integ.state(), y_eager), f"replay {rep}"
        assert np.array_equal(integ.cell_stats(), st_eager), f"replay {rep}"
    integ.close()


def test_lockstep_forcing_and_per_species_atol(oracle, parity):
    w = W.make_workload("s21_r84_262k", 96)
    rng = np.random.default_rng(12)
    F = rng.uniform(-1.0, 1.0, w["y0"].shape) * 1e2
    atol = np.geomspace(1e-12, 1e-9, 21)
    w = dict(w, F=F, atol=atol)
    import torch
    from paper_2405_01713_amd import bdfx
    integ = bdfx.Integrator(w["mechs"], w["y0"], w["rtol"], atol, T=w["T"], forcing=F,
                            scheduler=0, lockstep=4)
    integ.integrate(0.0, w["t_out"])
    torch.cuda.synchronize()
    y, st = integ.state(), integ.cell_stats()
    integ.close()
    yo, sto = oracle.integrate(w["mechs"], w["y0"], 0.0, w["t_out"], w["rtol"], atol, T=w["T"],
                               F=F, lockstep=4)
    assert np.all(st["status"] == 0) and np.all(sto["status"] == 0)
    parity(y, yo, w, "lock-step forcing")


def test_lockstep_reports_its_launch_shape():
    from paper_2405_01713_amd import bdfx
    w = W.make_workload("s21_r84_262k", 40)
    integ = bdfx.Integrator(w["mechs"], w["y0"], w["rtol"], w["atol"], T=w["T"], scheduler=1,
                            lockstep=4, waves_per_block=2, queue_chunk=4)
    for t in (integ.tuning(), integ.autotune(0.0, w["t_out"])):
        assert t[0]["waves_per_block"] == 4 and t[0]["cells_per_wave"] == 1
        assert t[0]["queue_chunk"] == 1 and t[0]["tables"] == 1 and t[0]["sample_cells"] == 0
    integ.close()


def test_lockstep_largest_batch_small_system(oracle, parity):
    """Robertson (3 species) in batches of 16 cells, the largest batch: 1,024
    threads per block; 100 cells leave a short last batch of 4."""
    w = W.make_workload("robertson_4k", 100)
    y, st = _gpu(w, lockstep=16, scheduler=1)
    yo, sto = _oracle(oracle, w, 16)
    assert np.all(st["status"] == 0) and np.all(sto["status"] == 0)
    parity(y, yo, w, "lock-step B16")
    nst = st["nst"]
    for k in range(0, 100, 16):
        assert np.all(nst[k:k + 16] == nst[k])
