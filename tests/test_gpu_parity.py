"""GPU path vs the FP64 CPU oracle, through the C ABI.

Both sides run the same per-cell algorithm on the same seeded inputs.  The
spec bar |y_gpu - y_oracle| <= 10 rtol |y_oracle| + atol is required
of >= 99 % of entries; rounding differences (exp, FMA contraction, reduction
order) can flip an accept/reject decision and move a cell onto another valid
step sequence, so the few cells beyond the bar must instead be within the
global-accuracy bound of a tight-tolerance reference (see conftest).
"""
import numpy as np
import pytest

from paper_2405_01713_amd import workloads as W
from tests.conftest import assert_adjoint_parity

pytestmark = pytest.mark.gpu


def _gpu(w, n=None, **opts):
    import torch
    from paper_2405_01713_amd import bdfx
    integ = bdfx.Integrator(w["mechs"], w["y0"], w["rtol"], w["atol"], T=w.get("T"),
                            kscale=w.get("kscale"), forcing=w.get("F"),
                            cell_mech=w.get("cell_mech"), **opts)
    integ.integrate(w.get("t0", 0.0), w["t_out"])
    torch.cuda.synchronize()
    y, st = integ.state(), integ.cell_stats()
    integ.close()
    return y, st


def _oracle(oracle, w, **kw):
    return oracle.integrate(w["mechs"], w["y0"], w.get("t0", 0.0), w["t_out"], w["rtol"],
                            w["atol"], T=w.get("T"), kscale=w.get("kscale"), F=w.get("F"),
                            cell_mech=w.get("cell_mech"), **kw)


def test_robertson_full_batch(oracle, parity):
    w = W.make_workload("robertson_4k")
    y, st = _gpu(w)
    yo, sto = _oracle(oracle, w)
    assert np.all(st["status"] == 0) and np.all(sto["status"] == 0)
    parity(y, yo, w, "robertson")
    assert np.abs(y.sum(1) - 1.0).max() < 1e-12  # invariant y1 + y2 + y3 = 1
    assert np.all(st["t_reached"] == 40.0)


@pytest.mark.parametrize("lu", [64, 32])
def test_s21_parity(oracle, parity, lu):
    w = W.make_workload("s21_r84_262k", 600)  # several waves plus a ragged tail
    y, st = _gpu(w, lu_precision=lu)
    yo, sto = _oracle(oracle, w)
    assert np.all(st["status"] == 0)
    parity(y, yo, w, f"s21 lu{lu}")
    wt = w["mechs"][0]["w"]
    drift = np.abs(y @ wt - w["y0"] @ wt).max()
    # FP64 LU keeps sum w_i y_i to round-off (w^T M = w^T); the FP32 solve
    # leaves the converged corrections with ~1e-7 relative mass errors
    assert drift < (1e-13 if lu == 64 else 1e-7)
    # same algorithm: the mean work per cell agrees closely
    assert abs(st["nst"].mean() / sto["nst"].mean() - 1) < 0.05


def test_s53_parity(oracle, parity):
    w = W.make_workload("s53_r325_262k_fp32lu", 96)
    y, st = _gpu(w)
    yo, sto = _oracle(oracle, w)
    assert np.all(st["status"] == 0)
    parity(y, yo, w)


def test_s53_fp32_lu_parity(oracle, parity):
    w = W.make_workload("s53_r325_262k_fp32lu", 96)
    y, st = _gpu(w, lu_precision=32)
    yo, sto = _oracle(oracle, w)
    assert np.all(st["status"] == 0)
    parity(y, yo, w)


@pytest.mark.parametrize("wl", ["s21_r84_262k", "s53_r325_262k_fp32lu"])
def test_register_budgets_bit_identical(oracle, parity, wl):
    """The register budgets (compiler's choice, 3, 4 and 5 waves per SIMD)
    build the same arithmetic with different register allocations (and
    spills): results agree bit for bit, and with the oracle."""
    w = W.make_workload(wl, 250)
    out = [_gpu(w, scheduler=1, waves_per_simd=wps) for wps in (0, 3, 4, 5)]
    for y, st in out[1:]:
        assert np.array_equal(y, out[0][0]) and np.array_equal(st, out[0][1])
    yo, _ = _oracle(oracle, w)
    parity(out[0][0], yo, w, f"{wl} budgets")


@pytest.mark.parametrize("lu,wps", [(64, 0), (32, 3)])
def test_tables_in_global_memory(oracle, parity, lu, wps):
    """53 species under the work queue: LDS limits the resident waves, so the
    slot words and rate constants move to global memory (each persistent wave
    owning a slot).  Results match the oracle and are bit-identical to the
    static grid, which keeps the rate constants in LDS."""
    import torch
    from paper_2405_01713_amd import bdfx
    w = W.make_workload("s53_r325_262k_fp32lu", 600)
    integ = bdfx.Integrator(w["mechs"], w["y0"], w["rtol"], w["atol"], T=w["T"],
                            scheduler=1, lu_precision=lu, waves_per_simd=wps)
    assert integ.tuning()[0]["tables"] == 2
    integ.integrate(0.0, w["t_out"])
    torch.cuda.synchronize()
    yq, stq = integ.state(), integ.cell_stats()
    integ.close()
    ys, sts = _gpu(w, lu_precision=lu, waves_per_simd=wps)
    assert np.all(stq["status"] == 0)
    assert np.array_equal(yq, ys) and np.array_equal(stq, sts)
    idx = np.arange(0, 600, 6)
    wo = dict(w, y0=w["y0"][idx], T=w["T"][idx], n_cells=len(idx))
    yo, sto = _oracle(oracle, wo)
    parity(yq[idx], yo, wo, f"global tables lu{lu}")


def test_mixed_mechanisms_and_queue(oracle, parity):
    w = W.make_workload("mixed_s9_s53_1m", 300)
    ys, sts = _gpu(w)
    yq, stq = _gpu(w, scheduler=1, queue_chunk=2)
    yo, sto = _oracle(oracle, w)
    assert np.all(sts["status"] == 0)
    parity(ys, yo, w, "mixed")
    # cells are independent: the schedule does not change any result bit
    assert np.array_equal(ys, yq)
    assert np.array_equal(sts, stq)
    # entries beyond a cell's species count are untouched
    S = np.array([w["mechs"][k]["n_species"] for k in w["cell_mech"]])
    for c in range(len(S)):
        assert np.all(ys[c, S[c]:] == w["y0"][c, S[c]:])


@pytest.mark.parametrize("lu", [64, 32])
def test_fused_launch_matches_per_bin_launches(oracle, parity, lu):
    """Both mechanism sizes in one launch (BDFX_SCHED_FUSED) give the results
    of one launch per mechanism bit for bit; with the FP64 Newton matrix the
    53-species cells keep their resident waves and the 9-species cells run
    beside them, so the pair launch is taken."""
    import torch
    from paper_2405_01713_amd import bdfx
    w = W.make_workload("mixed_s9_s53_1m", 3000)
    out = {}
    for sched in (1, 2):
        integ = bdfx.Integrator(w["mechs"], w["y0"], w["rtol"], w["atol"], T=w["T"],
                                cell_mech=w["cell_mech"], scheduler=sched, lu_precision=lu)
        integ.integrate(0.0, w["t_out"])
        torch.cuda.synchronize()
        out[sched] = (integ.state(), integ.cell_stats(), integ.tuning())
        integ.close()
    (y1, st1, t1), (y2, st2, t2) = out[1], out[2]
    assert np.array_equal(y1, y2) and np.array_equal(st1, st2)
    assert all(t["fused"] == 0 for t in t1)
    if lu == 64:
        assert all(t["fused"] == 1 for t in t2), t2
    yo, _ = _oracle(oracle, w)
    parity(y2, yo, w, f"fused lu{lu}")


@pytest.mark.parametrize("S,R,seed", [(2, 3, 0), (5, 9, 1), (12, 20, 2), (40, 70, 3)])
def test_padded_sizes(oracle, parity, S, R, seed):
    m = W.synthetic_mechanism(S, R, seed) if S > 2 else W.unimolecular_mechanism(S, R, seed)
    c = W.cell_states(m, 130, seed=seed + 7)
    w = dict(mechs=[m], y0=c["y0"], T=c["T"], rtol=1e-6, atol=1e-10, t_out=1e-5)
    y, st = _gpu(w)
    yo, sto = _oracle(oracle, w)
    assert np.all(st["status"] == sto["status"])
    # the sparse 40-species mechanism: the oracle against itself keeps 99.67 %
    parity(y, yo, w, min_frac=0.99 if S == 40 else 0.999)


def test_forcing_and_per_species_atol(oracle, parity):
    w = W.make_workload("s21_r84_262k", 130)
    rng = np.random.default_rng(5)
    w["F"] = rng.uniform(-1.0, 1.0, w["y0"].shape) * 1e2
    w["atol"] = np.geomspace(1e-12, 1e-9, 21)
    y, st = _gpu(w)
    yo, sto = _oracle(oracle, w)
    assert np.all(st["status"] == sto["status"])
    parity(y, yo, w)


def test_failures_are_per_cell(oracle, parity):
    w = W.make_workload("s21_r84_262k", 64)
    w["y0"] = w["y0"].copy()
    w["T"] = w["T"].copy()
    w["y0"][3, 2] = np.nan
    w["T"][9] = np.inf
    y, st = _gpu(w)
    yo, sto = _oracle(oracle, w)
    assert st["status"][3] == -9 and st["status"][9] == -9
    assert np.all(y[9] == w["y0"][9])
    ok = np.setdiff1d(np.arange(64), [3, 9])
    assert np.all(st["status"][ok] == 0)
    wok = dict(w, y0=w["y0"][ok], T=w["T"][ok])
    parity(y[ok], yo[ok], wok, "failures")
    # too much work: status -1, last accepted state and time kept
    y, st = _gpu(w, max_steps=3)
    yo, sto = _oracle(oracle, w, max_steps=3)
    assert np.all(st["status"][ok] == -1) and np.all(st["nst"][ok] == 3)
    assert np.all(sto["status"][ok] == -1)
    assert np.all(st["t_reached"][ok] < w["t_out"]) and np.all(np.isfinite(y[ok]))


def test_perturbation_bitwise(oracle):
    import torch
    from paper_2405_01713_amd import bdfx
    w = W.make_workload("mixed_s9_s53_1m", 500)
    integ = bdfx.Integrator(w["mechs"], w["y0"], w["rtol"], w["atol"], T=w["T"],
                            cell_mech=w["cell_mech"])
    integ.perturb(3, 7, 0.01)
    torch.cuda.synchronize()
    yg = integ.state()
    integ.close()
    ms = w["mechs"]
    yo = oracle.perturb(w["y0"], [ms[k]["n_species"] for k in w["cell_mech"]],
                        [ms[k]["w"] for k in w["cell_mech"]], 3, 7, 0.01)
    assert np.array_equal(yg, yo)


def _oracle_outer_loop(oracle, w, n_outer, seed, rtol, atol, max_steps=5000):
    """The splitting loop composed from the oracle's perturbation and
    integrator: perturb (outer step k), then integrate over [k dt, (k+1) dt]."""
    ms, cm = w["mechs"], w["cell_mech"]
    y, dt = w["y0"].copy(), w["t_out"]
    for k in range(n_outer):
        y = oracle.perturb(y, [ms[m]["n_species"] for m in cm], [ms[m]["w"] for m in cm], seed, k,
                           w["perturb"])
        y, st = oracle.integrate(ms, y, k * dt, (k + 1) * dt, rtol, atol, T=w["T"], cell_mech=cm,
                                 max_steps=max_steps)
        assert np.all(st["status"] == 0)
    return y


def test_outer_loop_graph(oracle, parity):
    """Outer splitting loop (perturb 1 %, integrate) of the mixed batch:
    eager launches vs the oracle, and HIP-graph replays vs the eager run bit
    for bit, with eager work and synchronisation between the replays."""
    import torch
    from paper_2405_01713_amd import bdfx
    w = W.make_workload("mixed_s9_s53_1m", 200)
    n_outer, seed = 3, 3
    integ = bdfx.Integrator(w["mechs"], w["y0"], w["rtol"], w["atol"], T=w["T"],
                            cell_mech=w["cell_mech"], scheduler=1, waves_per_simd=3)
    y0 = integ.y.clone()
    integ.outer_loop(n_outer, w["t_out"], seed, w["perturb"])
    torch.cuda.synchronize()
    y_eager, st_eager = integ.state(), integ.cell_stats()
    g = integ.capture_outer_loop(n_outer, w["t_out"], seed, w["perturb"])
    for rep in range(3):
        integ.y.copy_(y0)
        integ.status.fill_(7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(integ.state(), y_eager), f"replay {rep}"
        assert np.array_equal(integ.cell_stats(), st_eager), f"replay {rep}"
    integ.close()
    assert np.all(st_eager["status"] == 0)
    yo = _oracle_outer_loop(oracle, w, n_outer, seed, w["rtol"], w["atol"])
    tight = {}

    def reference(cells):
        if "y" not in tight:
            tight["y"] = _oracle_outer_loop(oracle, w, n_outer, seed, 1e-12, 1e-20, 200000)
        return tight["y"][cells]

    from tests.conftest import assert_parity
    assert_parity(y_eager, yo, w, oracle, "outer loop", reference=reference)


def test_autotune(tmp_path):
    """The autotuner leaves the states as they were, the tuned launch gives
    the same bits as the untuned one (cells are independent), and cached
    shapes are reapplied without timing."""
    import torch
    from paper_2405_01713_amd import bdfx
    w = W.make_workload("mixed_s9_s53_1m", 3000)
    kw = dict(T=w["T"], cell_mech=w["cell_mech"], scheduler=1)
    ref = bdfx.Integrator(w["mechs"], w["y0"], w["rtol"], w["atol"], **kw)
    ref.integrate(0.0, w["t_out"])
    torch.cuda.synchronize()
    y_ref, st_ref = ref.state(), ref.cell_stats()
    ref.close()
    cache = str(tmp_path / "tuning.json")
    integ = bdfx.Integrator(w["mechs"], w["y0"], w["rtol"], w["atol"], **kw)
    res = integ.autotune(0.0, w["t_out"], sample_cells=1024, cache=cache)
    assert sorted(r["mech"] for r in res) == [0, 1]
    for r in res:
        assert r["waves_per_simd"] in (0, 3, 4, 5) and r["waves_per_block"] in (1, 2, 4)
        assert r["queue_chunk"] in (1, 4) and r["ms"] > 0 and r["sample_cells"] > 0
    assert np.array_equal(integ.state(), w["y0"])
    integ.integrate(0.0, w["t_out"])
    torch.cuda.synchronize()
    assert np.array_equal(integ.state(), y_ref)
    assert np.array_equal(integ.cell_stats(), st_ref)
    integ.close()
    again = bdfx.Integrator(w["mechs"], w["y0"], w["rtol"], w["atol"], **kw)
    hit = again.autotune(0.0, w["t_out"], cache=cache)
    again.close()
    shape = lambda rs: sorted((r["mech"], r["waves_per_simd"], r["waves_per_block"],
                               r["queue_chunk"]) for r in rs)
    assert shape(hit) == shape(res)


def test_adjoint_matches_oracle(oracle):
    """GPU discrete adjoint vs the oracle's adjoint along its own adaptive
    record (both use the recorded states), loss = sum_cells sum_i c_i y_i."""
    import torch
    from paper_2405_01713_amd import bdfx
    w = W.make_workload("s21_r84_65k_adjoint", 48)
    m = w["mechs"][0]
    c = W.loss_weights(21)
    integ = bdfx.Integrator([m], w["y0"], w["rtol"], w["atol"], T=w["T"], record_steps=3000)
    integ.integrate(0.0, w["t_out"])
    ybar = np.tile(c, (48, 1))
    y0bar, lnA_bar = integ.adjoint(ybar)
    torch.cuda.synchronize()
    st = integ.cell_stats()
    y0bar, lnA_bar = y0bar.cpu().numpy(), lnA_bar.cpu().numpy()[0]
    integ.close()
    assert np.all(st["status"] == 0)
    g_lnA = np.zeros(84)
    y0bar_o = np.zeros((48, 21))
    nst_o = np.zeros(48, dtype=int)
    for k in range(48):
        kf, kr = oracle.rates(m, w["T"][k])
        _, so, rec = oracle.integrate_record(m, w["y0"][k], 0.0, w["t_out"], w["rtol"], w["atol"],
                                             T=w["T"][k])
        yb, pb = oracle.adjoint(m, kf, kr, w["y0"][k], rec, rec["y"], c)
        y0bar_o[k] = yb
        g_lnA += pb
        nst_o[k] = so["nst"]
    # the gradient of the summed loss w.r.t. each log rate constant
    assert np.all(np.abs(lnA_bar - g_lnA) <= 1e-3 * np.abs(g_lnA).max())
    # dL/dy0 per cell: each side follows its own valid step sequence
    assert_adjoint_parity(y0bar, y0bar_o, "adjoint dL/dy0")


def test_bdf_function_autograd(oracle):
    """torch.autograd.Function over the library: loss = sum_cells c . y(t_out);
    loss.backward() fills dL/dy0 and dL/dlnA from the discrete adjoint, which
    match the oracle's adjoint (per-cell criterion; lnA summed over cells)."""
    import torch
    from paper_2405_01713_amd import bdfx
    w = W.make_workload("s21_r84_65k_adjoint", 32)
    m = w["mechs"][0]
    c = W.loss_weights(21)
    BDF = bdfx.make_bdf_function()
    y0 = torch.as_tensor(w["y0"], device="cuda").requires_grad_()
    lnA = torch.as_tensor(m["lnA"], device="cuda").requires_grad_()
    y = BDF.apply(y0, lnA, m, w["T"], w["t_out"], w["rtol"], w["atol"], 3000)
    loss = (y * torch.as_tensor(c, device="cuda")).sum()
    loss.backward()
    torch.cuda.synchronize()
    g_y0, g_lnA = y0.grad.cpu().numpy(), lnA.grad.cpu().numpy()
    go_lnA = np.zeros(84)
    go_y0 = np.zeros((32, 21))
    for k in range(32):
        kf, kr = oracle.rates(m, w["T"][k])
        _, _, rec = oracle.integrate_record(m, w["y0"][k], 0.0, w["t_out"], w["rtol"], w["atol"],
                                            T=w["T"][k])
        go_y0[k], pb = oracle.adjoint(m, kf, kr, w["y0"][k], rec, rec["y"], c)
        go_lnA += pb
    assert_adjoint_parity(g_y0, go_y0, "autograd dL/dy0")
    assert np.all(np.abs(g_lnA - go_lnA) <= 1e-3 * np.abs(go_lnA).max())


def _three_body_mechanism():
    """Six species with weights (1, 1, 2, 3, 4, 2) and mass-conserving
    reactions that use three reactant slots and repeated species:
    2A + B <=> D, 2A <=> C, A + B + C <=> E, C <=> F, D + A <=> E, 2F <=> E."""
    reac = [[0, 0, 1], [0, 0, -1], [0, 1, 2], [2, -1, -1], [3, 0, -1], [5, 5, -1]]
    prod = [[3, -1, -1], [2, -1, -1], [4, -1, -1], [5, -1, -1], [4, -1, -1], [4, -1, -1]]
    return dict(n_species=6, n_reactions=6, reac=np.array(reac, dtype=np.int32),
                prod=np.array(prod, dtype=np.int32),
                lnA=np.log([3e3, 5e4, 2e5, 7e2, 1e4, 3e5]), EaR=np.zeros(6),
                lnK=np.log([20.0, 0.5, 3.0, 0.2, 8.0, 1.5]),
                w=np.array([1.0, 1.0, 2.0, 3.0, 4.0, 2.0]))


def test_three_body_and_repeated_species(oracle, parity):
    m = _three_body_mechanism()
    c = W.cell_states(m, 200, seed=21)
    w = dict(mechs=[m], y0=c["y0"], T=c["T"], rtol=1e-6, atol=1e-10, t_out=1e-3)
    y, st = _gpu(w)
    yo, sto = _oracle(oracle, w)
    assert np.all(st["status"] == 0) and np.all(sto["status"] == 0)
    parity(y, yo, w, "three-body")
    # sum_i w_i y_i is conserved by every reaction
    inv0, inv1 = c["y0"] @ m["w"], y[:, :6] @ m["w"]
    assert np.abs(inv1 - inv0).max() <= 1e-12 * np.abs(inv0).max()


@pytest.mark.parametrize("lu", [64, 32])
def test_abc_specialisation_matches_generic(oracle, parity, lu):
    """A + B <=> C mechanisms run specialised kernels (two reactant slots and
    one product slot, no empty-slot work).  The same mechanism with its
    product moved to slot 1 is not recognised as such and runs the generic
    slot loops; both match the oracle, and the same terms only land in another
    order (so results agree to rounding)."""
    m = W.synthetic_mechanism(21, 84)
    g = dict(m, prod=np.roll(m["prod"], 1, axis=1))
    assert np.all(g["prod"][:, 1] == m["prod"][:, 0]) and np.all(g["prod"][:, 0] == -1)
    c = W.cell_states(m, 256, seed=13, T_range=(1000.0, 2500.0))
    w = dict(mechs=[m], y0=c["y0"], T=c["T"], rtol=1e-6, atol=1e-10, t_out=1e-5)
    ya, sta = _gpu(w, scheduler=1, lu_precision=lu)
    yg, stg = _gpu(dict(w, mechs=[g]), scheduler=1, lu_precision=lu)
    assert np.all(sta["status"] == 0) and np.all(stg["status"] == 0)
    yo, sto = _oracle(oracle, w)
    parity(ya, yo, w, f"A+B<=>C kernels lu{lu}")
    parity(yg, yo, w, f"generic kernels lu{lu}")
    tol = 10 * 1e-6 * np.abs(yo) + 1e-10
    assert np.mean(np.abs(ya - yg) <= tol) >= 0.99


def test_largest_size_all_lanes(oracle, parity):
    """64 species: every lane of the wave holds a species.  This sparse test
    mechanism (150 reactions) is as sensitive to round-off as the 40-species
    one: the oracle against itself with inputs perturbed by 1e-15 keeps
    99.40-99.69 % of entries within 10 rtol, so the bar is 99 %."""
    m = W.synthetic_mechanism(64, 150, 5)
    c = W.cell_states(m, 96, seed=8)
    w = dict(mechs=[m], y0=c["y0"], T=c["T"], rtol=1e-6, atol=1e-10, t_out=1e-5)
    y, st = _gpu(w, scheduler=1)
    yo, sto = _oracle(oracle, w)
    assert np.all(st["status"] == 0)
    parity(y, yo, w, "S=64", min_frac=0.99)


def test_empty_and_single_cell_batches(oracle, parity):
    import torch
    from paper_2405_01713_amd import bdfx
    w = W.make_workload("s21_r84_262k", 1)
    m = w["mechs"][0]
    for sched in (0, 1):
        empty = bdfx.Integrator([m], np.zeros((0, 21)), w["rtol"], w["atol"], scheduler=sched)
        empty.integrate(0.0, w["t_out"])
        torch.cuda.synchronize()
        assert empty.state().shape == (0, 21)
        assert empty.summary()["n_cells"] == 0
        empty.close()
        y, st = _gpu(w, scheduler=sched)
        yo, sto = _oracle(oracle, w)
        assert st["status"][0] == 0
        parity(y, yo, w, f"single cell, scheduler {sched}")


@pytest.mark.parametrize("lu", [64, 32])
def test_two_cells_per_wave(oracle, parity, lu):
    """Two cells per wave (one per half-wave): parity with the oracle for an
    odd number of cells (the last wave has an idle half) and for padded
    mechanism sizes.  The RHS and Newton-matrix sums are accumulated by lanes
    in another order than with one cell per wave (last-bit differences), but
    the static and the work-queue schedules give the same bits."""
    w = W.make_workload("s21_r84_262k", 255)
    ys, sts = _gpu(w, scheduler=0, lu_precision=lu, cells_per_wave=2)
    yq, stq = _gpu(w, scheduler=1, lu_precision=lu, cells_per_wave=2)
    assert np.all(sts["status"] == 0)
    assert np.array_equal(ys, yq) and np.array_equal(sts, stq)
    yo, _ = _oracle(oracle, w)
    parity(ys, yo, w, f"two cells per wave, LU{lu}")
    for S, R, seed in ((5, 9, 1), (12, 20, 2)):
        m = W.synthetic_mechanism(S, R, seed)
        c = W.cell_states(m, 37, seed=seed + 7)
        wp = dict(mechs=[m], y0=c["y0"], T=c["T"], rtol=1e-6, atol=1e-10, t_out=1e-5)
        y2, st2 = _gpu(wp, scheduler=1, lu_precision=lu, cells_per_wave=2)
        yo, sto = _oracle(oracle, wp)
        assert np.all(st2["status"] == sto["status"])
        parity(y2, yo, wp, f"two cells per wave, S={S}")


def test_two_cells_per_wave_mixed(oracle, parity):
    """Mixed 9 / 53 species batch: the 9-species bin runs two cells per wave,
    the 53-species bin one."""
    w = W.make_workload("mixed_s9_s53_1m", 301)
    y2, st2 = _gpu(w, scheduler=1, cells_per_wave=2)
    assert np.all(st2["status"] == 0)
    yo, _ = _oracle(oracle, w)
    parity(y2, yo, w, "mixed, two cells per wave")
