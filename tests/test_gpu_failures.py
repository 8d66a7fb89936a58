"""Per-cell failures on the GPU, forced from the host, and schedule independence.

Each failure status is produced on the device without any kernel misbehaving:
a limit on error-test failures (-3) or Newton convergence failures (-4) per
step, an exactly singular Newton matrix (-6), a full step record (-10).  The
contract checked each time (the paper's accept/reject logic, Sec. 2: a step
that is not accepted leaves the solution unchanged; cells are independent,
Sec. 4.1.1): a failed cell keeps its last accepted state and time -- those of
a run stopped after the same number of accepted steps (bit for bit, or up to
the rounding of the restored prediction when the failure came within a step)
-- and every other cell is bit-identical to a run in which nothing failed.
"""
import numpy as np
import pytest

from paper_2405_01713_amd import workloads as W

pytestmark = pytest.mark.gpu


def _gpu(w, **opts):
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


def _stopped_after(w, cells, nst, y, st, exact=True, **opts):
    """Failed cells keep the state and time of a run stopped (status -1) after
    the same number of accepted steps.  A cell that failed within a step
    attempt has its Nordsieck array restored by the inverse of the prediction,
    which is exact up to rounding (1e-13 of the cell's largest entry);
    otherwise the states are equal bit for bit."""
    for n in np.unique(nst[cells])[:4]:
        sel = cells[nst[cells] == n]
        ys, sts = _gpu(w, max_steps=int(n), **opts) if n > 0 else (w["y0"], None)
        if exact:
            assert np.array_equal(y[sel], ys[sel]), n
        else:
            tol = 1e-13 * np.abs(ys[sel]).max(axis=1, keepdims=True)
            assert np.all(np.abs(y[sel] - ys[sel]) <= tol), n
        if sts is not None:
            assert np.all(sts["status"][sel] == -1)
            assert np.array_equal(st["t_reached"][sel], sts["t_reached"][sel])


# Whether a cell ever meets `limit` failures within one step depends on its
# exact step sequence, which round-off moves: the oracle against itself with
# inputs perturbed by 1e-15 fails the same cells for 90.6-92.0 % of cells
# (error tests, 21 species, limit 2) and 98.0-98.2 % (convergence, the mixed
# 9/53-species batch, limit 1).  The bars sit three binomial standard
# deviations (512 cells) below the worst of those.  The 21-species workload
# has no convergence failures at all, so that case runs the mixed batch.
@pytest.mark.parametrize("kind,option,code,workload,agree_min", [
    ("error test", "max_err_test_fails", -3, "s21_r84_262k", 0.86),
    ("convergence", "max_conv_fails", -4, "mixed_s9_s53_1m", 0.96)])
def test_failure_limits_per_step(oracle, kind, option, code, workload, agree_min):
    w = W.make_workload(workload, 512)
    y_ref, st_ref = _gpu(w, scheduler=1)
    counter = "netf" if code == -3 else "ncfn"
    assert np.all(st_ref["status"] == 0) and st_ref[counter].sum() > 0
    # the smallest limit at which some cells fail and some do not
    for lim in range(1, 8):
        y, st = _gpu(w, scheduler=1, **{option: lim})
        failed = np.nonzero(st["status"] != 0)[0]
        if 0 < failed.size < 512:
            break
    else:
        pytest.fail(f"no {kind} limit splits the batch")
    ok = np.setdiff1d(np.arange(512), failed)
    assert np.all(st["status"][failed] == code)
    assert np.all(st["t_reached"][failed] < w["t_out"])
    # the others never reached the limit: bit-identical to the unlimited run
    assert np.array_equal(y[ok], y_ref[ok]) and np.array_equal(st[ok], st_ref[ok])
    _stopped_after(w, failed, st["nst"], y, st, exact=False, scheduler=1)
    # the oracle with the same limit fails the same cells (round-off may move
    # a cell with an exactly borderline count)
    yo, sto = oracle.integrate(w["mechs"], w["y0"], 0.0, w["t_out"], w["rtol"], w["atol"],
                               T=w["T"], cell_mech=w.get("cell_mech"),
                               **{("max_netf" if code == -3 else "max_ncf"): lim})
    agree = np.mean(st["status"] == sto["status"])
    assert agree >= agree_min, agree
    assert np.all(np.isin(sto["status"], (0, code)))


def _autocatalytic():
    """A -> 2A and B -> 2B with rate constants exp(0) * kscale = 2^20 and 2^22
    (exact), from y = 0.  f(0) = 0, so the initial step is the upper bound
    0.1 (t_out - t0), which is exactly 2^-20 for t_out - t0 = 10 * 2^-20; at
    order 1 gamma = h, so M = I - gamma J = diag(1 - 1, 1 - 4) is exactly
    singular, and again diag(1 - 1/4, 1 - 1) after the step is cut by 4 --
    in either precision -- and the cell fails with -6 before any step."""
    return dict(n_species=2, n_reactions=2,
                reac=np.array([[0, -1, -1], [1, -1, -1]], dtype=np.int32),
                prod=np.array([[0, 0, -1], [1, 1, -1]], dtype=np.int32),
                lnA=np.zeros(2), EaR=np.zeros(2), lnK=None, w=np.ones(2))


@pytest.mark.parametrize("lu", [64, 32])
def test_singular_newton_matrix(oracle, lu):
    base = W.make_workload("s21_r84_262k", 96)
    t_out = 10.0 * 2.0 ** -20
    sing = _autocatalytic()
    cm = np.zeros(96, dtype=np.int32)
    cm[::5] = 1
    sc = cm == 1
    y0 = base["y0"].copy()
    y0[sc] = 0.0
    ks = np.ones((96, 84))
    ks[sc, 0], ks[sc, 1] = 2.0 ** 20, 2.0 ** 22
    T = base["T"].copy()
    T[sc] = 1.0
    w = dict(mechs=[base["mechs"][0], sing], y0=y0, T=T, kscale=ks, cell_mech=cm, rtol=1e-6,
             atol=1e-10, t_out=t_out)
    y, st = _gpu(w, lu_precision=lu)
    assert np.all(st["status"][sc] == -6) and np.all(st["nst"][sc] == 0)
    assert np.all(st["nsetups"][sc] == 2) and np.all(st["t_reached"][sc] == 0.0)
    assert np.all(y[sc] == 0.0)
    # the other cells are bit-identical to a batch without the singular ones
    ok = ~sc
    wo = dict(base, y0=base["y0"][ok], T=base["T"][ok], kscale=ks[ok], t_out=t_out)
    y_ok, st_ok = _gpu(wo, lu_precision=lu)
    assert np.all(st_ok["status"] == 0)
    assert np.array_equal(y[ok, :21], y_ok) and np.array_equal(st[ok], st_ok)
    # the oracle takes the same path
    yo, sto = oracle.integrate([sing], y0[sc][:, :2], 0.0, t_out, 1e-6, 1e-10, T=T[sc],
                               kscale=ks[sc][:, :2])
    assert np.all(sto["status"] == -6) and np.all(sto["nsetups"] == 2) and np.all(yo == 0.0)



@pytest.mark.parametrize("lu", [64, 32])
def test_singular_newton_matrix_in_a_large_kernel(oracle, lu):
    """The same two autocatalytic reactions among 19 species (17 of them
    inert: unit rows of the Newton matrix), so the cells run the 21-species
    kernels, whose FP64 pivot search takes its second (low-word) pass only
    when the largest high word is tied: an all-zero column ties every lane
    and must still be found singular.  Every cell fails with -6 before any
    step, as in the oracle, with its state untouched."""
    sing = _autocatalytic()
    S = 19
    m = dict(sing, n_species=S, w=np.ones(S))
    n = 64
    rng = np.random.default_rng(5)
    y0 = np.zeros((n, S))
    y0[:, 2:] = rng.uniform(0.1, 1.0, size=(n, S - 2))
    ks = np.ones((n, 2))
    ks[:, 0], ks[:, 1] = 2.0 ** 20, 2.0 ** 22
    T = np.ones(n)
    t_out = 10.0 * 2.0 ** -20
    w = dict(mechs=[m], y0=y0, T=T, kscale=ks, rtol=1e-6, atol=1e-10, t_out=t_out)
    y, st = _gpu(w, lu_precision=lu)
    assert np.all(st["status"] == -6) and np.all(st["nst"] == 0)
    assert np.all(st["nsetups"] == 2) and np.all(st["t_reached"] == 0.0)
    assert np.array_equal(y[:, :S], y0)
    yo, sto = oracle.integrate([m], y0[:8], 0.0, t_out, 1e-6, 1e-10, T=T[:8], kscale=ks[:8])
    assert np.all(sto["status"] == -6) and np.all(sto["nsetups"] == 2)
    assert np.array_equal(yo, y0[:8])

def test_record_capacity(oracle):
    """A cell that needs more accepted steps than the record holds fails with
    -10 at its last recorded step: the returned state is the record's last
    state, the time is the sum of the recorded steps; cells within the
    capacity are bit-identical to a run without recording."""
    from paper_2405_01713_amd import bdfx
    import torch
    w = W.make_workload("s21_r84_65k_adjoint", 64)
    y_ref, st_ref = _gpu(w)
    cap = int(np.median(st_ref["nst"]))
    integ = bdfx.Integrator(w["mechs"], w["y0"], w["rtol"], w["atol"], T=w["T"], record_steps=cap)
    integ.integrate(0.0, w["t_out"])
    torch.cuda.synchronize()
    y, st = integ.state(), integ.cell_stats()
    recs = integ.step_record(np.arange(64))
    integ.close()
    full = st_ref["nst"] > cap
    assert full.any() and (~full).any()
    assert np.all(st["status"][full] == -10) and np.all(st["nst"][full] == cap)
    assert np.all(st["status"][~full] == 0)
    assert np.array_equal(y[~full], y_ref[~full]) and np.array_equal(st[~full], st_ref[~full])
    for c in np.nonzero(full)[0]:
        assert recs[c]["n"] == cap
        assert np.array_equal(y[c], recs[c]["y"][-1])
        assert st["t_reached"][c] == pytest.approx(recs[c]["h"].sum(), rel=1e-13)
    _stopped_after(w, np.nonzero(full)[0], st["nst"], y, st)
    # the oracle with the same capacity stops its cells at the same point
    # (cells clear of the capacity: round-off moves step counts by a few)
    _, sto = oracle.integrate(w["mechs"], w["y0"], 0.0, w["t_out"], w["rtol"], w["atol"], T=w["T"])
    clear = np.nonzero(full & (st_ref["nst"] > 1.05 * cap) & (sto["nst"] > 1.05 * cap))[0]
    assert clear.size >= 4
    for c in clear[:4]:
        yo, so, _ = oracle.integrate_record(w["mechs"][0], w["y0"][c], 0.0, w["t_out"], w["rtol"],
                                            w["atol"], T=w["T"][c], cap=cap)
        assert so["status"] == -10 and so["nst"] == cap
        # the two runs stop at different times (their step sequences differ by
        # round-off); the GPU's state is the solution at its own stopping time,
        # within the global-accuracy envelope of 100 error weights
        yt, _ = oracle.integrate(w["mechs"], w["y0"][c:c + 1], 0.0, float(st["t_reached"][c]),
                                 w["rtol"], w["atol"], T=w["T"][c:c + 1])
        assert np.all(np.abs(yt[0] - y[c]) <= 100 * (w["rtol"] * np.abs(yt[0]) + w["atol"]))


@pytest.mark.parametrize("scheduler", [0, 1])
def test_cell_permutation_bitwise(scheduler):
    """Chemistry is local to each cell (Sec. 4.1.1): integrating the cells in
    another order permutes the results and changes no bit, for a mixed batch
    of two mechanism sizes under either scheduler."""
    w = W.make_workload("mixed_s9_s53_1m", 700)
    y, st = _gpu(w, scheduler=scheduler)
    perm = np.random.default_rng(9).permutation(700)
    wp = dict(w, y0=w["y0"][perm], T=w["T"][perm], cell_mech=w["cell_mech"][perm])
    yp, stp = _gpu(wp, scheduler=scheduler)
    assert np.array_equal(yp, y[perm])
    assert np.array_equal(stp, st[perm])
