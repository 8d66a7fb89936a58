"""Checkpointed step records for the adjoint (bdfx_options.checkpoint_every).

With checkpoint_every = K > 0 the forward run keeps, instead of every accepted
step, the integrator's whole state at every K-th step; bdfx_adjoint() reruns
each K-step segment from its checkpoint with the same step code and sweeps it
backwards.  The rerun takes the same steps to the bit, so the gradient must
equal the full record's exactly: compared bit for bit here for several K (one
step per segment, K dividing nothing, one segment for the whole run), on one
mechanism and on a two-mechanism batch (per-bin launches and the one-launch
form), on 4,096 cells whose segment counts differ (each pass covers those
cells that still have a segment), and when the record fills up.
The forward results do not depend on the recording mode either.
"""
import numpy as np
import pytest

from paper_2405_01713_amd import workloads as W

pytestmark = pytest.mark.gpu


def _grad(w, ybar, **opts):
    from paper_2405_01713_amd import bdfx
    integ = bdfx.Integrator(w["mechs"], w["y0"], w["rtol"], w["atol"], T=w["T"],
                            cell_mech=w["cell_mech"], **opts)
    integ.integrate(0.0, w["t_out"])
    y0bar, lnA_bar = integ.adjoint(ybar)
    out = dict(y=np.array(integ.state()), st=integ.cell_stats(), y0bar=y0bar.cpu().numpy(),
               lnA_bar=lnA_bar.cpu().numpy(), ws=integ.ws_bytes)
    if not opts.get("checkpoint_every"):
        out["recs"] = integ.step_record(np.arange(min(len(w["y0"]), 64)))
    integ.close()
    return out


def _ybar(w):
    n = len(w["y0"])
    ldy = max(int(m["n_species"]) for m in w["mechs"])
    yb = np.zeros((n, ldy))
    cm = np.zeros(n, dtype=np.int64) if w["cell_mech"] is None else np.asarray(w["cell_mech"])
    for k, m in enumerate(w["mechs"]):
        S = int(m["n_species"])
        yb[cm == k, :S] = W.loss_weights(S)
    return yb


def _same(a, b, what):
    assert np.array_equal(a["y"], b["y"]), f"{what}: forward states differ"
    for k in ("status", "nst", "nfe", "nsetups", "netf", "ncfn", "q_last"):
        assert np.array_equal(a["st"][k], b["st"][k]), f"{what}: stats {k} differ"
    assert np.array_equal(a["y0bar"], b["y0bar"]), (
        f"{what}: dL/dy0 differs, worst {np.abs(a['y0bar'] - b['y0bar']).max():.3g}")
    assert np.array_equal(a["lnA_bar"], b["lnA_bar"]), f"{what}: dL/dlnA differs"


def test_checkpointed_gradient_equals_the_full_record_bit_for_bit():
    w = W.make_workload("s21_r84_65k_adjoint", 64)
    yb = _ybar(w)
    full = _grad(w, yb, record_steps=3000)
    assert np.all(full["st"]["status"] == 0)
    nst = full["st"]["nst"]
    # the runs hold order changes in both directions and step-size changes
    q = np.concatenate([r["q"] for r in full["recs"]])
    assert q.min() == 1 and q.max() >= 4
    print(f"steps per cell {nst.min()}..{nst.max()}, "
          f"rebuilt steps {sum(int(r['rebuild'].sum()) for r in full['recs'])}")
    ws = {}
    for K in (1, 7, 32, 3000):
        ck = _grad(w, yb, record_steps=3000, checkpoint_every=K)
        _same(full, ck, f"K={K}")
        ws[K] = ck["ws"]
        print(f"K={K}: workspace {ck['ws'] / 2**20:.1f} MiB vs {full['ws'] / 2**20:.1f} MiB")
    # checkpoints of 20 + 8 S doubles every 32 steps instead of S + 2 per step
    assert ws[32] * 3 < full["ws"]


@pytest.mark.parametrize("scheduler", [1, 2])
def test_checkpointed_gradient_two_mechanisms(scheduler):
    """The 9- and 53-species mechanisms of the mixed workload; scheduler 2 runs
    both bins in one launch (the checkpoints are written by that kernel)."""
    w = W.make_workload("mixed_s9_s53_1m", 96)
    yb = _ybar(w)
    full = _grad(w, yb, record_steps=1500, scheduler=scheduler)
    assert np.all(full["st"]["status"] == 0)
    ck = _grad(w, yb, record_steps=1500, scheduler=scheduler, checkpoint_every=16)
    _same(full, ck, f"scheduler {scheduler}")


def test_checkpointed_sweep_on_4096_cells():
    """4,096 cells in segments of 24 steps; their step counts differ by many
    segments, so the later passes rerun and sweep only the cells with the most
    steps."""
    w = W.make_workload("s21_r84_65k_adjoint", 4096)
    yb = _ybar(w)
    full = _grad(w, yb, record_steps=2048, scheduler=1)
    nst = full["st"]["nst"]
    print(f"steps per cell {nst.min()}..{nst.max()}")
    assert np.all(full["st"]["status"] == 0) and nst.max() - nst.min() >= 10 * 24
    ck = _grad(w, yb, record_steps=2048, scheduler=1, checkpoint_every=24)
    _same(full, ck, "4096 cells")
    assert ck["ws"] * 2 < full["ws"]  # 188 doubles per 24 steps instead of 23 per step


def test_checkpointed_record_that_fills_up():
    """record_steps = 40, not a multiple of K = 16: cells with more steps stop
    at step 40 with BDFX_CELL_RECORD_FULL, and the gradient is that of the
    recorded map, as with the full record."""
    from paper_2405_01713_amd import bdfx
    w = W.make_workload("s21_r84_65k_adjoint", 64)
    yb = _ybar(w)
    full = _grad(w, yb, record_steps=40)
    st = full["st"]
    assert np.any(st["status"] == bdfx.BDFX_CELL_RECORD_FULL)
    assert np.all(st["nst"][st["status"] == bdfx.BDFX_CELL_RECORD_FULL] == 40)
    ck = _grad(w, yb, record_steps=40, checkpoint_every=16)
    _same(full, ck, "record full")


def test_checkpoint_option_errors():
    from paper_2405_01713_amd import bdfx
    w = W.make_workload("s21_r84_65k_adjoint", 8)
    args = (w["mechs"], w["y0"], w["rtol"], w["atol"])
    for opts, code in ((dict(checkpoint_every=8), bdfx.BDFX_EINVAL),
                       (dict(checkpoint_every=-1, record_steps=64), bdfx.BDFX_EINVAL),
                       (dict(checkpoint_every=8, record_steps=64, lu_precision=32),
                        bdfx.BDFX_EUNSUPPORTED),
                       (dict(checkpoint_every=8, record_steps=64, jacobian=bdfx.BDFX_JAC_DQ),
                        bdfx.BDFX_EUNSUPPORTED)):
        with pytest.raises(bdfx.BdfxError, match=f"bdfx error {code}:"):
            bdfx.Integrator(*args, T=w["T"], **opts)
    integ = bdfx.Integrator(*args, T=w["T"], record_steps=64, checkpoint_every=8,
                            cells_per_wave=2)
    try:
        # two cells per wave is not used with checkpoints
        assert all(t["cells_per_wave"] == 1 for t in integ.tuning())
        integ.integrate(0.0, w["t_out"])
        with pytest.raises(bdfx.BdfxError, match=f"bdfx error {bdfx.BDFX_EUNSUPPORTED}:"):
            integ.step_record([0])
    finally:
        integ.close()
