"""Benchmark: cells integrated per second per outer step (one MI355X).

Headline workload: 1,048,576 cells, half with the 9-species / 30-reaction and
half with the 53-species / 325-reaction synthetic mass-action mechanism
(T ~ U[800, 2800] K), ten outer splitting steps of 1e-5 s, each a 1 %
perturbation of the states followed by the integration of every cell, all ten
captured in one HIP graph; rtol = 1e-6, atol = 1e-10, FP64 throughout, the
persistent work-queue form with autotuned launch shapes, one launch per
mechanism per outer step ("batched").  One bench step is one outer step; K steps are timed as graph replays from the resident
initial state (K/10 replays of the ten-step graph, plus one graph of K mod 10
steps), with HIP events on the replay stream.

Also measured (labelled keys, each with its own small step count): the same
workload with both mechanism sizes in one launch ("batched_fused"), with the
FP32 Newton matrix and in the plain (static grid) form; the
21-species workload on 262,144 cells in the three forms; the 53-species
mechanism on 262,144 cells (FP64 vs FP32 Newton matrix) and on 1,048,576 cells;
the discrete adjoint on 65,536 cells; and the CPU oracle on a random sample of
the headline workload.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2405_01713_amd import workloads as W  # noqa: E402

FP64_VECTOR_PEAK_TFLOPS = 78.6
FP32_VECTOR_PEAK_TFLOPS = 157.3
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def kernel_source_hash() -> str:
    """Hash of the HIP sources and build flags; a stored traffic figure is
    reported only while this matches."""
    import hashlib
    from paper_2405_01713_amd import build as B
    # flags without the checkout's location, so that copies of the tree agree
    h = hashlib.sha256(" ".join(f.replace(B.ROOT, "<root>") for f in B.CFLAGS).encode())
    csrc = os.path.join(ROOT, "paper_2405_01713_amd", "csrc")
    files = [os.path.join(csrc, f) for f in sorted(os.listdir(csrc)) if f.endswith((".hip", ".h"))]
    files.append(os.path.join(ROOT, "include", "bdfx.h"))
    for path in files:
        with open(path, "rb") as fh:
            h.update(os.path.basename(path).encode() + fh.read())
    return h.hexdigest()[:16]


def _pmc_rows(d):
    import csv
    import glob
    rows = []
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            rows += list(csv.DictReader(fh))
    return rows


def traffic_from(fetch_dir, write_dir, copy_mib, workload, form, out=TRAFFIC_FILE):
    """HBM traffic of the integrator launches of one outer step from two
    rocprofv3 --pmc runs of ``bench.py --pmc-step --copy-probe copy_mib``
    (FETCH_SIZE, then WRITE_SIZE; KiB per dispatch): the k_integrate
    dispatches after the probe copy are summed.  Each counter is scaled by its
    reading for the probe copy, which reads and writes copy_mib MiB."""
    res = {}
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = [r for r in _pmc_rows(d) if r["Counter_Name"] == counter]
        by = {}
        for r in rows:
            k = int(r["Dispatch_Id"])
            by.setdefault(k, [r["Kernel_Name"], 0.0])[1] += float(r["Counter_Value"])
        copies = [(k, v) for k, v in sorted(by.items()) if "bdfx" not in v[0]]
        k_copy, (_, copy_kib) = max(copies, key=lambda kv: kv[1][1])
        # the integrator launches after the probe: those of the measured step
        integ = [v for k, v in sorted(by.items()) if "k_integrate" in v[0] and k > k_copy]
        kib = sum(v[1] for v in integ)
        factor = copy_mib * 1024.0 / copy_kib
        res[counter] = dict(integrate_kib=kib, launches=len(integ), copy_kib=copy_kib,
                            scale=factor, bytes=kib * factor * 1024.0)
    doc = dict(workload=workload, form=form, source_hash=kernel_source_hash(), copy_mib=copy_mib,
               fetch=res["FETCH_SIZE"], write=res["WRITE_SIZE"],
               traffic_bytes=res["FETCH_SIZE"]["bytes"] + res["WRITE_SIZE"]["bytes"])
    with open(out, "w") as fh:
        json.dump(doc, fh, indent=1)
    return doc


def stored_traffic(workload, form):
    try:
        with open(TRAFFIC_FILE) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    if d.get("workload") != workload or d.get("form") != form:
        return None
    return d["traffic_bytes"] if d.get("source_hash") == kernel_source_hash() else None




# ---------------------------------------------------------------------------
# algorithmic flops
# ---------------------------------------------------------------------------

def flops_per_cell(S: int, R: int, st: np.ndarray, fp32_lu: bool = False) -> tuple:
    """Algorithmic flops of one integration of each cell in ``st`` (per-cell
    statistics of a mechanism with S species and R reactions), counted from
    the cell's own event counters (FMA = 2, divide / sqrt / exp = 1):

        F = nfe 7R + nsetups (11R + S^2 + 2S^3/3) + nni (2S^2 + 8S)
            + nst (q^2/2 + 2q + 12) S + R (4 + 1)

    (right-hand sides; Jacobian, Newton matrix and LU factorisation per setup;
    solve and vector work per Newton iteration; predictor, correction, norms
    and rescaling per step at order q; rate constants with one exp each).  q is
    the cell's last order.  Returns (FP64 flops, FP32 flops) per cell; with the
    FP32 Newton matrix the factorisation and the solves are FP32."""
    nfe, nst, nni, nsu = (st[k].astype(np.float64) for k in ("nfe", "nst", "nni", "nsetups"))
    q = st["q_last"].astype(np.float64)
    lu, solve = 2.0 * S ** 3 / 3.0, 2.0 * S * S
    total = (nfe * 7 * R + nsu * (11 * R + S * S + lu) + nni * (solve + 8 * S)
             + nst * (q * q / 2 + 2 * q + 12) * S + R * 5)
    f32 = nsu * lu + nni * solve if fp32_lu else np.zeros_like(total)
    return total - f32, f32


def launch_flops(w, st, fp32_lu=False) -> tuple:
    """(FP64, FP32) algorithmic flops summed over the cells of a launch."""
    cm = w["cell_mech"] if w.get("cell_mech") is not None else np.zeros(len(st), dtype=int)
    F64 = F32 = 0.0
    for k, m in enumerate(w["mechs"]):
        sel = cm == k
        if sel.any():
            a, b = flops_per_cell(int(m["n_species"]), int(m["n_reactions"]), st[sel], fp32_lu)
            F64 += float(a.sum())
            F32 += float(b.sum())
    return F64, F32


def roofline_frac(F64, F32, seconds):
    """Fraction of the vector peaks: F64 / t / 78.6 TF + F32 / t / 157.3 TF."""
    return (F64 / seconds / (FP64_VECTOR_PEAK_TFLOPS * 1e12)
            + F32 / seconds / (FP32_VECTOR_PEAK_TFLOPS * 1e12))


FORM_OPTS = dict(plain=dict(scheduler=0, lu_precision=64),
                 batched=dict(scheduler=1, lu_precision=64),
                 batched_fused=dict(scheduler=2, lu_precision=64),
                 batched_fp32lu=dict(scheduler=1, lu_precision=32))


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# ---------------------------------------------------------------------------
# headline: the outer splitting loop in a HIP graph
# ---------------------------------------------------------------------------

def run_outer_loop(w, form, steps, warmup, tuning_cache=None, seed=3, account=True):
    """Time exactly ``steps`` outer steps of the workload (graphs of 10 outer
    steps replayed from the resident initial state, plus one graph of
    steps mod 10), after ``warmup`` untimed outer steps run the same way.
    With ``account``, one more eager pass of the ten outer steps from the same
    state reads every step's per-cell statistics (algorithmic flops) and times
    each integrator launch with HIP events on the launch stream; its final
    state must equal the graph's bit for bit."""
    import torch
    from paper_2405_01713_amd import bdfx

    n_outer, dt, amp = w["outer_steps"], w["t_out"], w["perturb"]
    integ = bdfx.Integrator(w["mechs"], w["y0"], w["rtol"], w["atol"], T=w["T"],
                            kscale=w["kscale"], cell_mech=w["cell_mech"], **FORM_OPTS[form])
    tuning = integ.autotune(0.0, dt, cache=tuning_cache) if FORM_OPTS[form]["scheduler"] else None
    y0 = integ.y.clone()
    graphs = {}

    def graph(n):
        if n not in graphs:
            graphs[n] = integ.capture_outer_loop(n, dt, seed, amp)
        return graphs[n]

    def plan(total):
        return [n_outer] * (total // n_outer) + ([total % n_outer] if total % n_outer else [])

    stream = torch.cuda.current_stream()
    for n in plan(warmup):
        integ.y.copy_(y0)
        graph(n).replay()
    torch.cuda.synchronize()
    times = []
    wall0 = time.perf_counter()
    for n in plan(steps):
        integ.y.copy_(y0)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        graph(n).replay()
        b.record(stream)
        times.append((n, a, b))
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms = [(n, a.elapsed_time(b)) for n, a, b in times]
    total_ms = sum(t for _, t in ms)
    # state after one full graph of n_outer steps from y0 (for the oracle check)
    integ.y.copy_(y0)
    graph(n_outer).replay()
    torch.cuda.synchronize()
    y_graph = integ.state()
    st_last = integ.cell_stats()
    out = dict(form=form, outer_steps_timed=steps, replays=[n for n, _ in ms],
               replay_ms=[t for _, t in ms], ms_per_outer_step=total_ms / steps,
               wall_ms_per_outer_step=1e3 * wall / steps,
               cells_per_s=w["n_cells"] * steps / (total_ms * 1e-3), tuning=tuning,
               failed_cells_last_step=int(np.sum(st_last["status"] != 0)))
    if account:
        integ.y.copy_(y0)
        F64 = F32 = 0.0
        launch_ms, failed = [], 0
        per_mech_nst = {}
        with torch.cuda.stream(integ.stream):
            for k in range(n_outer):
                integ.perturb(seed, k, amp)
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record(integ.stream)
                integ.integrate(k * dt, (k + 1) * dt)
                b.record(integ.stream)
                torch.cuda.synchronize()
                launch_ms.append(a.elapsed_time(b))
                st = integ.cell_stats()
                failed += int(np.sum(st["status"] != 0))
                f64, f32 = launch_flops(w, st, form == "batched_fp32lu")
                F64 += f64
                F32 += f32
                for m in range(len(w["mechs"])):
                    key = f"S{w['mechs'][m]['n_species']}"
                    nst = st["nst"][w["cell_mech"] == m] if w["cell_mech"] is not None else st["nst"]
                    per_mech_nst.setdefault(key, []).append(float(nst.mean()))
        y_eager = integ.state()
        out.update(alg_flops_fp64_per_outer_step=F64 / n_outer,
                   alg_flops_fp32_per_outer_step=F32 / n_outer,
                   eager_integrate_ms=launch_ms, eager_integrate_ms_mean=float(np.mean(launch_ms)),
                   failed_cell_steps=failed, mean_nst_per_outer_step=per_mech_nst,
                   graph_equals_eager_bitwise=bool(np.array_equal(y_graph, y_eager)))
    integ.close()
    out["_y"] = y_graph
    return out


# ---------------------------------------------------------------------------
# single-step forms (21-species workload)
# ---------------------------------------------------------------------------

def run_form(w, form, steps, warmup, tuning_cache=None):
    """One outer step of every cell from the same resident state (restored by
    a device copy before each step), timed with HIP events on the launch
    stream; ``steps`` timed after ``warmup``."""
    import torch
    from paper_2405_01713_amd import bdfx

    opts = FORM_OPTS[form]
    integ = bdfx.Integrator(w["mechs"], w["y0"], w["rtol"], w["atol"], T=w["T"],
                            kscale=w["kscale"], cell_mech=w["cell_mech"], **opts)
    tuning = (integ.autotune(0.0, w["t_out"], cache=tuning_cache) if opts["scheduler"] == 1
              else None)
    y0 = integ.y.clone()
    stream = integ.stream
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    with torch.cuda.stream(stream):
        for _ in range(warmup):
            integ.y.copy_(y0)
            integ.integrate(0.0, w["t_out"])
        torch.cuda.synchronize()
        for k in range(steps):
            integ.y.copy_(y0)
            ev[k][0].record(stream)
            integ.integrate(0.0, w["t_out"])
            ev[k][1].record(stream)
        torch.cuda.synchronize()
    kern_ms = [a.elapsed_time(b) for a, b in ev]
    y = integ.state()
    st = integ.cell_stats()
    integ.close()
    F64, F32 = launch_flops(w, st, form == "batched_fp32lu")
    t = float(np.mean(kern_ms)) * 1e-3
    return dict(kernel_ms=float(np.mean(kern_ms)), kernel_ms_min=float(np.min(kern_ms)),
                cells_per_s=w["n_cells"] / t, alg_flops_fp64=F64, alg_flops_fp32=F32,
                roofline_frac=roofline_frac(F64, F32, t),
                failed_cells=int(np.sum(st["status"] != 0)), mean_nst=float(st["nst"].mean()),
                mean_nsetups=float(st["nsetups"].mean()), tuning=tuning,
                min_y=float(y.min()), n_below_minus_atol=int(np.sum(y < -np.asarray(w["atol"]))),
                invariant_drift=_invariant_drift(w, y), _y=y)


def run_c1(steps, warmup, tuning_cache=None, n_check=256):
    """The 21-species / 84-reaction workload on 262,144 cells in the three
    forms; the first n_check cells against the oracle."""
    w = W.make_workload("s21_r84_262k")
    out = dict(workload="s21_r84_262k", n_cells=w["n_cells"])
    ys = {}
    for form in ("plain", "batched", "batched_fp32lu"):
        r = run_form(w, form, steps, warmup, tuning_cache)
        ys[form] = r.pop("_y")[:n_check]
        out[form] = r
        log(f"21 species {form}: {r['kernel_ms']:.1f} ms")
    try:
        from oracle import oracle as O
        yo, _ = O.integrate(w["mechs"], w["y0"][:n_check], 0.0, w["t_out"], w["rtol"], w["atol"],
                            T=w["T"][:n_check])
        for form in ys:
            out[form]["vs_oracle"] = _errors(ys[form], yo, w["rtol"], w["atol"])
        out["check_cells"] = n_check
    except Exception as e:  # the oracle is optional on the timing path
        out["check_error"] = repr(e)
    return out


def run_adjoint(steps, warmup, n_cells=None, record_steps=2048, n_check=32, ckpt_every=128):
    """Adjoint/forward cost on the 65,536-cell 21-species workload: plain
    forward (no recording), forward with step recording, discrete-adjoint
    backward of the loss sum_cells sum_i c_i y_i; a sample of cells is checked
    against the oracle's adjoint along the GPU's own step record (the same
    frozen map, so the two differ by round-off).  Then the same with
    checkpointed records (a checkpoint every ckpt_every steps, segments rerun
    in the backward sweep): its workspace, times, and whether its gradient
    equals the full record's bit for bit."""
    import torch
    from paper_2405_01713_amd import bdfx

    w = W.make_workload("s21_r84_65k_adjoint", n_cells)
    m, N = w["mechs"][0], w["n_cells"]
    c = W.loss_weights(m["n_species"])
    ybar = torch.as_tensor(np.tile(c, (N, 1)), device="cuda")

    def timed(fn, stream):
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(steps)]
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        for k in range(steps):
            ev[k][0].record(stream)
            fn()
            ev[k][1].record(stream)
        torch.cuda.synchronize()
        return float(np.median([a.elapsed_time(b) for a, b in ev]))

    common = dict(scheduler=1)
    plain = bdfx.Integrator([m], w["y0"], w["rtol"], w["atol"], T=w["T"], **common)
    tune = plain.autotune(0.0, w["t_out"])
    common.update(waves_per_simd=tune[0]["waves_per_simd"],
                  waves_per_block=tune[0]["waves_per_block"], queue_chunk=tune[0]["queue_chunk"])
    y0 = plain.y.clone()

    def fwd_plain():
        plain.y.copy_(y0)
        plain.integrate(0.0, w["t_out"])

    t_fwd = timed(fwd_plain, plain.stream)
    plain.close()
    rec = bdfx.Integrator([m], w["y0"], w["rtol"], w["atol"], T=w["T"],
                          record_steps=record_steps, **common)

    def fwd_rec():
        rec.y.copy_(y0)
        rec.integrate(0.0, w["t_out"])

    t_rec = timed(fwd_rec, rec.stream)
    out = {}

    def bwd():
        out["g"] = rec.adjoint(ybar)

    t_bwd = timed(bwd, rec.stream)
    log(f"adjoint: forward {t_fwd:.1f} ms, backward {t_bwd:.1f} ms")
    st = rec.cell_stats()
    g_full = [t.clone() for t in out["g"]]
    y0bar = g_full[0][:n_check].cpu().numpy()
    recs = rec.step_record(np.arange(n_check))
    ws_full = rec.ws_bytes
    rec.close()
    res = dict(workload="s21_r84_65k_adjoint", n_cells=N, fwd_ms=t_fwd, fwd_record_ms=t_rec,
               bwd_ms=t_bwd, ratio_bwd_over_fwd=t_bwd / t_fwd,
               ratio_fwd_record_plus_bwd_over_fwd=(t_rec + t_bwd) / t_fwd,
               failed_cells=int(np.sum(st["status"] != 0)), max_nst=int(st["nst"].max()),
               workspace_full_record_mb=ws_full / 1e6)

    ck = bdfx.Integrator([m], w["y0"], w["rtol"], w["atol"], T=w["T"], record_steps=record_steps,
                         checkpoint_every=ckpt_every, **common)

    def fwd_ck():
        ck.y.copy_(y0)
        ck.integrate(0.0, w["t_out"])

    t_fck = timed(fwd_ck, ck.stream)

    def bwd_ck():
        out["gc"] = ck.adjoint(ybar)

    t_bck = timed(bwd_ck, ck.stream)
    torch.cuda.synchronize()
    res["checkpointed"] = dict(
        every=ckpt_every, workspace_mb=ck.ws_bytes / 1e6, fwd_ms=t_fck, bwd_ms=t_bck,
        ratio_bwd_over_fwd=t_bck / t_fwd, ratio_fwd_plus_bwd_over_fwd=(t_fck + t_bck) / t_fwd,
        workspace_ratio_full_over_checkpointed=ws_full / ck.ws_bytes,
        gradient_bitwise_equal=bool(torch.equal(out["gc"][0], g_full[0]) and
                                    torch.equal(out["gc"][1], g_full[1])))
    ck.close()
    log(f"checkpointed adjoint (every {ckpt_every}): forward {t_fck:.1f} ms, backward "
        f"{t_bck:.1f} ms, workspace {ws_full / 1e6:.0f} -> {res['checkpointed']['workspace_mb']:.0f} MB")
    try:
        from oracle import oracle as O
        go = np.zeros((n_check, m["n_species"]))
        for k in range(n_check):
            kf, kr = O.rates(m, w["T"][k])
            r = recs[k]
            go[k] = O.adjoint(m, kf, kr, r["y0"], r, r["y"], c)[0]
        rel = np.abs(y0bar[:, :m["n_species"]] - go).max(axis=1) / np.abs(go).max(axis=1)
        res["check_cells"] = n_check
        res["check_worst_rel"] = float(rel.max())
        res["check_median_rel"] = float(np.median(rel))
        # the GPU test's bar for dL/dy0 along the GPU record (3e-10 per cell)
        res["check_ok"] = bool(rel.max() <= 3e-10)
    except Exception as e:  # the oracle is optional on the timing path
        res["check_error"] = repr(e)
    return res


def _timed_events(fn, stream, steps, warmup):
    import torch
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    for k in range(steps):
        ev[k][0].record(stream)
        fn()
        ev[k][1].record(stream)
    torch.cuda.synchronize()
    return float(np.median([a.elapsed_time(b) for a, b in ev]))


def _invariant_drift(w, y):
    """max over cells of |sum_i w_i y_i - sum_i w_i y0_i| (species weights of
    each cell's mechanism)."""
    cm = w["cell_mech"] if w.get("cell_mech") is not None else np.zeros(len(y), dtype=int)
    drift = 0.0
    for k, m in enumerate(w["mechs"]):
        sel = cm == k
        S = m["n_species"]
        d = np.abs(y[sel, :S] @ m["w"] - w["y0"][sel, :S] @ m["w"])
        drift = max(drift, float(d.max()) if d.size else 0.0)
    return drift


def _errors(y, yo, rtol, atol):
    """max |dy| / (|y_o| + atol) and max |dy| / (rtol |y_o| + atol) (error-weight units)."""
    dy = np.abs(y - yo)
    return dict(max_rel_err=float(np.max(dy / (np.abs(yo) + atol))),
                max_err_units=float(np.max(dy / (rtol * np.abs(yo) + atol))),
                frac_within_10rtol=float(np.mean(dy <= 10 * rtol * np.abs(yo) + atol)))


def run_precision(steps, warmup, tuning_cache=None, n_cells=None, n_check=256):
    """53 species / 325 reactions on 262,144 cells (or n_cells): FP64 vs FP32
    Newton-matrix inverse, both through the autotuned work queue; errors of
    both against the FP64 oracle on the first n_check cells."""
    from paper_2405_01713_amd import bdfx

    w = W.make_workload("s53_r325_262k_fp32lu", n_cells)
    label = "s53_r325_1m" if w["n_cells"] == 1 << 20 else "s53_r325_262k_fp32lu"
    out = dict(workload=label, n_cells=w["n_cells"])
    ys = {}
    for lu in (64, 32):
        integ = bdfx.Integrator(w["mechs"], w["y0"], w["rtol"], w["atol"], T=w["T"], scheduler=1,
                                lu_precision=lu)
        tune = integ.autotune(0.0, w["t_out"], cache=tuning_cache)
        y0 = integ.y.clone()

        def step():
            integ.y.copy_(y0)
            integ.integrate(0.0, w["t_out"])

        ms = _timed_events(step, integ.stream, steps, warmup)
        st = integ.cell_stats()
        ys[lu] = integ.state()[:n_check]
        integ.close()
        log(f"precision lu{lu}: {ms:.1f} ms")
        F64, F32 = launch_flops(w, st, lu == 32)
        out[f"lu{lu}"] = dict(kernel_ms=ms, cells_per_s=w["n_cells"] / (ms * 1e-3), tuning=tune,
                              failed_cells=int(np.sum(st["status"] != 0)),
                              mean_nst=float(st["nst"].mean()),
                              mean_nsetups=float(st["nsetups"].mean()),
                              alg_flops_fp64=F64, alg_flops_fp32=F32,
                              roofline_frac=roofline_frac(F64, F32, ms * 1e-3))
    out["speedup_fp32lu_over_fp64"] = out["lu64"]["kernel_ms"] / out["lu32"]["kernel_ms"]
    try:
        from oracle import oracle as O
        yo, _ = O.integrate(w["mechs"], w["y0"][:n_check], 0.0, w["t_out"], w["rtol"], w["atol"],
                            T=w["T"][:n_check])
        for lu in (64, 32):
            out[f"lu{lu}"]["vs_oracle"] = _errors(ys[lu], yo, w["rtol"], w["atol"])
        out["check_cells"] = n_check
    except Exception as e:  # the oracle is optional on the timing path
        out["check_error"] = repr(e)
    return out


def run_thermal(tuning_cache=None, n_cells=None, n_check=128):
    """Non-isothermal cells: the 21-species mechanism with synthetic
    thermochemistry, temperature as the 22nd state entry, 262,144 cells, one
    outer step; batched (work queue, autotuned) with the FP64 and the FP32
    Newton matrix, against the isothermal run of the same states; the first
    n_check cells checked against the oracle with the global-error bar."""
    from paper_2405_01713_amd import bdfx

    w = W.make_workload("s21_r84_thermal_262k", n_cells)
    out = dict(workload="s21_r84_thermal_262k", n_cells=w["n_cells"])
    ys = {}
    for lu in (64, 32):
        integ = bdfx.Integrator(w["mechs"], w["y0"], w["rtol"], w["atol"], scheduler=1,
                                lu_precision=lu)
        tune = integ.autotune(0.0, w["t_out"], cache=tuning_cache)
        y0 = integ.y.clone()

        def step():
            integ.y.copy_(y0)
            integ.integrate(0.0, w["t_out"])

        ms = _timed_events(step, integ.stream, 1, 1)
        st = integ.cell_stats()
        ys[lu] = integ.state()[:n_check]
        integ.close()
        log(f"thermal lu{lu}: {ms:.1f} ms")
        out[f"lu{lu}"] = dict(kernel_ms=ms, cells_per_s=w["n_cells"] / (ms * 1e-3), tuning=tune,
                              failed_cells=int(np.sum(st["status"] != 0)),
                              mean_nst=float(st["nst"].mean()), mean_nfe=float(st["nfe"].mean()))
    try:
        from oracle import oracle as O
        sub = dict(w, y0=w["y0"][:n_check], n_cells=n_check)
        yo, _ = O.integrate(w["mechs"], sub["y0"], 0.0, w["t_out"], w["rtol"], w["atol"])
        for lu in (64, 32):
            out[f"lu{lu}"]["vs_oracle"] = _errors(ys[lu], yo, w["rtol"], w["atol"])
        out["check_cells"] = n_check
    except Exception as e:  # the oracle is optional on the timing path
        out["check_error"] = repr(e)
    return out


def run_dq(tuning_cache=None, n_check=128):
    """Newton matrix from difference quotients (Table 1, approaches 3A/3B)
    against the analytic Jacobian on the 21-species workload (262,144 cells,
    one outer step, work queue, FP32 Newton matrix): time, right-hand sides
    per cell, and the first n_check cells against the oracle run with
    difference quotients."""
    from paper_2405_01713_amd import bdfx

    w = W.make_workload("s21_r84_262k")
    out = dict(workload="s21_r84_262k", n_cells=w["n_cells"])
    ys = None
    for name, jac in (("analytic", bdfx.BDFX_JAC_ANALYTIC), ("dq", bdfx.BDFX_JAC_DQ)):
        integ = bdfx.Integrator(w["mechs"], w["y0"], w["rtol"], w["atol"], T=w["T"], scheduler=1,
                                lu_precision=32, jacobian=jac, waves_per_simd=4)
        y0 = integ.y.clone()

        def step():
            integ.y.copy_(y0)
            integ.integrate(0.0, w["t_out"])

        ms = _timed_events(step, integ.stream, 1, 1)
        st = integ.cell_stats()
        if jac == bdfx.BDFX_JAC_DQ:
            ys = integ.state()[:n_check]
        integ.close()
        log(f"jacobian {name}: {ms:.1f} ms")
        out[name] = dict(kernel_ms=ms, cells_per_s=w["n_cells"] / (ms * 1e-3),
                         mean_nfe=float(st["nfe"].mean()), mean_nsetups=float(st["nsetups"].mean()),
                         mean_nst=float(st["nst"].mean()), failed_cells=int(np.sum(st["status"] != 0)))
    out["dq_over_analytic"] = out["dq"]["kernel_ms"] / out["analytic"]["kernel_ms"]
    try:
        from oracle import oracle as O
        yo, _ = O.integrate(w["mechs"], w["y0"][:n_check], 0.0, w["t_out"], w["rtol"], w["atol"],
                            T=w["T"][:n_check], jac_dq=True)
        out["dq"]["vs_oracle"] = _errors(ys, yo, w["rtol"], w["atol"])
        out["check_cells"] = n_check
    except Exception as e:  # the oracle is optional on the timing path
        out["check_error"] = repr(e)
    return out


def run_gmres(tuning_cache=None, n_check=128, t_out=1e-8, steps=3, warmup=1):
    """Inexact Newton with matrix-free GMRES (Table 1, approaches 1A/1B)
    against the direct solve (2A, FP64 and FP32 Newton matrix) on 262,144
    cells of the 21-species mechanism over an outer step of PeleC size
    (t_out = 1e-8 s), all on the autotuned work queue: time per outer step,
    work per cell, and the first n_check cells against an rtol = 1e-12 oracle
    reference (the forms differ in accuracy as well as speed) and against the
    oracle run with the same linear solver."""
    from paper_2405_01713_amd import bdfx

    w = dict(W.make_workload("s21_r84_262k"), t_out=t_out)
    out = dict(workload="s21_r84_262k", n_cells=w["n_cells"], t_out=t_out)
    forms = (("direct_fp64", dict(lu_precision=64)), ("direct_fp32", dict(lu_precision=32)),
             ("gmres5", dict(gmres_maxl=5)), ("gmres10", dict(gmres_maxl=10)))
    ys = {}
    for name, o in forms:
        integ = bdfx.Integrator(w["mechs"], w["y0"], w["rtol"], w["atol"], T=w["T"], scheduler=1,
                                **o)
        tuning = integ.autotune(0.0, t_out, cache=tuning_cache)
        y0 = integ.y.clone()

        def step():
            integ.y.copy_(y0)
            integ.integrate(0.0, t_out)

        ms = _timed_events(step, integ.stream, steps, warmup)
        st = integ.cell_stats()
        ys[name] = integ.state()[:n_check]
        integ.close()
        log(f"gmres leg {name}: {ms:.2f} ms")
        out[name] = dict(kernel_ms=ms, cells_per_s=w["n_cells"] / (ms * 1e-3),
                         mean_nst=float(st["nst"].mean()), mean_nfe=float(st["nfe"].mean()),
                         mean_nni=float(st["nni"].mean()), mean_nli=float(st["nli"].mean()),
                         mean_ncfl=float(st["ncfl"].mean()),
                         mean_nsetups=float(st["nsetups"].mean()),
                         failed_cells=int(np.sum(st["status"] != 0)), tuning=tuning)
    for name in ("gmres5", "gmres10"):
        out[f"{name}_over_direct_fp64"] = out[name]["kernel_ms"] / out["direct_fp64"]["kernel_ms"]
    try:
        from oracle import oracle as O
        sub = lambda a: a[:n_check]
        yr, _ = O.integrate(w["mechs"], sub(w["y0"]), 0.0, t_out, 1e-12, 1e-20, T=sub(w["T"]),
                            max_steps=500000)
        unit = w["rtol"] * np.abs(yr) + w["atol"]
        for name, o in forms:
            e = np.abs(ys[name] - yr) / unit
            out[name]["vs_tight_reference"] = dict(
                median_units=float(np.median(e)), p99_units=float(np.percentile(e, 99)),
                max_units=float(e.max()))
            if "gmres_maxl" in o:
                yo, _ = O.integrate(w["mechs"], sub(w["y0"]), 0.0, t_out, w["rtol"], w["atol"],
                                    T=sub(w["T"]), gmres_maxl=o["gmres_maxl"])
                out[name]["vs_oracle"] = _errors(ys[name], yo, w["rtol"], w["atol"])
        out["check_cells"] = n_check
    except Exception as e:  # the oracle is optional on the timing path
        out["check_error"] = repr(e)
    return out


def run_lockstep(tuning_cache=None, n_check=128, batches=(2, 4, 8), steps=3, warmup=1):
    """Per-cell step control against the paper's lock-step batches (Sec. 2:
    the cells of a batch share one step size and one WRMS norm) on the
    21-species workload (262,144 cells, one outer step, FP32 Newton matrix,
    work queue): time per outer step and accepted steps per cell, and the
    first n_check cells against the oracle run with the same batches."""
    from paper_2405_01713_amd import bdfx

    w = W.make_workload("s21_r84_262k")
    out = dict(workload="s21_r84_262k", n_cells=w["n_cells"])
    ys = {}
    for B in (0,) + tuple(batches):
        name = "per_cell" if B == 0 else f"batch{B}"
        integ = bdfx.Integrator(w["mechs"], w["y0"], w["rtol"], w["atol"], T=w["T"], scheduler=1,
                                lu_precision=32, lockstep=B)
        tuning = integ.autotune(0.0, w["t_out"], cache=tuning_cache) if B == 0 else None
        y0 = integ.y.clone()

        def step():
            integ.y.copy_(y0)
            integ.integrate(0.0, w["t_out"])

        ms = _timed_events(step, integ.stream, steps, warmup)
        st = integ.cell_stats()
        ys[B] = integ.state()[:n_check]
        integ.close()
        log(f"lockstep leg {name}: {ms:.1f} ms")
        out[name] = dict(kernel_ms=ms, cells_per_s=w["n_cells"] / (ms * 1e-3),
                         mean_nst=float(st["nst"].mean()), mean_nfe=float(st["nfe"].mean()),
                         mean_nsetups=float(st["nsetups"].mean()),
                         failed_cells=int(np.sum(st["status"] != 0)), tuning=tuning)
    for B in batches:
        out[f"batch{B}_over_per_cell"] = out[f"batch{B}"]["kernel_ms"] / out["per_cell"]["kernel_ms"]
    try:
        from oracle import oracle as O
        sub = lambda a: a[:n_check]
        for B in batches:
            yo, _ = O.integrate(w["mechs"], sub(w["y0"]), 0.0, w["t_out"], w["rtol"], w["atol"],
                                T=sub(w["T"]), lockstep=B)
            out[f"batch{B}"]["vs_oracle"] = _errors(ys[B], yo, w["rtol"], w["atol"])
        out["check_cells"] = n_check
    except Exception as e:  # the oracle is optional on the timing path
        out["check_error"] = repr(e)
    return out


def run_typical(tuning_cache=None, reps=50, eta=1e-10):
    """Typical-value absolute tolerances (Sec. 4.1.3): the device min/max pass
    over the states (HBM-bound; bytes = cells x species x 8 read) timed with
    HIP events on the 21-species workload and on 1,048,576 cells of the
    53-species mechanism, checked bit for bit against the oracle; then one
    outer step of the 21-species workload integrated with those tolerances
    (batched, FP32 Newton matrix) against the same run with atol = 1e-10."""
    import torch
    from paper_2405_01713_amd import bdfx

    out = {}
    for name, n in (("s21_r84_262k", None), ("s53_r325_262k_fp32lu", 1 << 20)):
        w = W.make_workload(name, n)
        S = w["mechs"][0]["n_species"]
        integ = bdfx.Integrator(w["mechs"], w["y0"], w["rtol"], w["atol"], T=w["T"], scheduler=1)
        typ = torch.empty((1, integ.S_max), dtype=torch.float64, device=integ.dev)
        ms = _timed_events(lambda: integ.typical_atol(eta, typ), integ.stream, reps, 5)
        nbytes = w["n_cells"] * S * 8
        t_host = typ.cpu().numpy()
        d = dict(n_cells=w["n_cells"], species=S, ms=ms, bytes=nbytes,
                 gb_per_s=nbytes / (ms * 1e-3) / 1e9, frac_hbm=nbytes / (ms * 1e-3) / 8.0e12)
        try:
            from oracle import oracle as O
            to, _ = O.typical_atol(w["y0"], eta, [S])
            d["bit_exact_vs_oracle"] = bool(np.array_equal(t_host, to[:, :integ.S_max]))
        except Exception as e:  # the oracle is optional on the timing path
            d["check_error"] = repr(e)
        integ.close()
        out[name if n is None else f"{name}@{n}"] = d
        log(f"typical {name}: {ms * 1e3:.1f} us, {d['gb_per_s']:.0f} GB/s")
    w = W.make_workload("s21_r84_262k")
    for mode in ("fixed", "typical"):
        integ = bdfx.Integrator(w["mechs"], w["y0"], w["rtol"], w["atol"], T=w["T"], scheduler=1,
                                lu_precision=32)
        integ.autotune(0.0, w["t_out"], cache=tuning_cache)
        y0 = integ.y.clone()

        def step():
            integ.y.copy_(y0)
            if mode == "typical":
                integ.typical_atol(eta)
            integ.integrate(0.0, w["t_out"])

        ms = _timed_events(step, integ.stream, 1, 1)
        st = integ.cell_stats()
        integ.close()
        out[f"integrate_{mode}"] = dict(ms=ms, cells_per_s=w["n_cells"] / (ms * 1e-3),
                                        mean_nst=float(st["nst"].mean()),
                                        failed_cells=int(np.sum(st["status"] != 0)))
        log(f"typical: integrate with {mode} atol {ms:.1f} ms")
    return out


# ---------------------------------------------------------------------------
# CPU oracle baseline
# ---------------------------------------------------------------------------

def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def _native_oracle():
    """Build the oracle with -O3 -march=native (same source, no FMA
    contraction, so its results equal the -O2 build's) into a temporary
    directory on this host; returns the library path."""
    import subprocess
    import tempfile
    from oracle import oracle as O
    d = tempfile.mkdtemp(prefix="bdfx_oracle_native_")
    path = os.path.join(d, "liboracle_native.so")
    subprocess.run(["gcc", "-O3", "-march=native", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                    "-ffp-contract=off", "-o", path, O.SRC, "-lm"], check=True)
    return path


def cpu_baseline(w, n_sample=4096, n_single=128, reps=3, seed=11, pert_seed=3):
    """The oracle on the GPU machine's host cores, on a random sample of the
    workload's cells (seeded): the whole outer loop (every outer step's
    perturbation, untimed, then the integration of the sample, timed), built
    with -O3 -march=native and OpenMP over all threads; median of ``reps``
    runs, plus one run on one thread over the first n_single cells of the
    sample.  cells/s per outer step = cells x outer steps / integration time."""
    from oracle import oracle as O

    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(w["n_cells"], size=min(n_sample, w["n_cells"]), replace=False))
    n_outer = w["outer_steps"]
    cm = w["cell_mech"][idx] if w["cell_mech"] is not None else np.zeros(idx.size, dtype=np.int32)
    T = None if w["T"] is None else w["T"][idx]

    def run(sel, threads):
        secs = []
        y, st = O.outer_loop(w["mechs"], w["y0"][idx[sel]], idx[sel], cm[sel], n_outer,
                             w["t_out"], pert_seed, w["perturb"], w["rtol"], w["atol"],
                             T=None if T is None else T[sel], integrate_seconds=secs,
                             nthreads=threads)
        return y, st, sum(secs)

    path = _native_oracle()
    all_sel = np.arange(idx.size)
    with O.use_library(path):
        threads = O.max_threads()
        times, y = [], None
        for _ in range(reps):
            y, st, t = run(all_sel, threads)
            times.append(t)
        t1 = run(all_sel[:n_single], 1)[2]
        O.set_threads(threads)
    # the -O2 oracle gives the same numbers (no FMA contraction in either build)
    y2, _ = O.outer_loop(w["mechs"], w["y0"][idx[:16]], idx[:16], cm[:16], 1, w["t_out"],
                         pert_seed, w["perturb"], w["rtol"], w["atol"],
                         T=None if T is None else T[:16])
    with O.use_library(path):
        y3, _ = O.outer_loop(w["mechs"], w["y0"][idx[:16]], idx[:16], cm[:16], 1, w["t_out"],
                             pert_seed, w["perturb"], w["rtol"], w["atol"],
                             T=None if T is None else T[:16])
    med = float(np.median(times))
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = os.cpu_count()
    return dict(value=idx.size * n_outer / med, unit="cells/s", cores=threads, kind="oracle",
                sample=(f"{idx.size} random cells (seed {seed}) of the {w['n_cells']} of the same "
                        f"workload, all {n_outer} outer steps (perturbation untimed), oracle "
                        f"built -O3 -march=native, OpenMP over {threads} threads; median of "
                        f"{reps} runs ({med:.1f} s)"),
                seconds=times, single_thread=dict(cells=int(min(n_single, idx.size)),
                                                  seconds=t1,
                                                  value=min(n_single, idx.size) * n_outer / t1),
                cpu_model=_cpu_model(), nproc=os.cpu_count(), affinity=affinity,
                native_equals_O2_build=bool(np.array_equal(y2, y3)),
                _idx=idx, _y=y)


def parity_summary(y, yo, rtol, atol):
    """Fraction of entries within 10 rtol |y_oracle| + atol, the worst entry
    over that bar, and the worst in units of 100 error weights."""
    err = np.abs(y - yo)
    r10 = err / (10 * rtol * np.abs(yo) + atol)
    r100 = err / (100 * (rtol * np.abs(yo) + atol))
    frac = float(np.mean(r10 <= 1.0))
    return dict(frac_within_10rtol=frac, worst_over_10rtol=float(r10.max()),
                worst_over_100_weights=float(r100.max()),
                parity_ok=bool(frac >= 0.99 and r100.max() <= 1.0))


# ---------------------------------------------------------------------------

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10, help="timed outer steps of the headline")
    ap.add_argument("--warmup", type=int, default=10, help="untimed outer steps before them")
    ap.add_argument("--cells", type=int, default=None, help="fewer headline cells (testing)")
    ap.add_argument("--cpu-sample", type=int, default=4096)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the headline workload's FP32-LU and plain forms")
    ap.add_argument("--no-c1", action="store_true", help="skip the 21-species legs")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the 53-species legs (262,144 and 1,048,576 cells)")
    ap.add_argument("--extra", default="",
                    help="comma list of longer measurements: 'typical' (typical-value "
                         "tolerances: reduction bandwidth and integration), 'thermal' (262,144 "
                         "non-isothermal 21-species cells), 'dq' (difference-quotient vs "
                         "analytic Jacobian), 'gmres' (matrix-free GMRES vs the direct solve over "
                         "a 1e-8 s outer step), 'lockstep' (per-cell step control vs lock-step "
                         "batches of 2, 4 and 8 cells)")
    ap.add_argument("--tuning-cache", default=None,
                    help="JSON file of autotuned launch shapes (reused when present)")
    ap.add_argument("--copy-probe", type=float, default=0.0,
                    help="first run a device copy of this many MiB (traffic scale reference)")
    ap.add_argument("--pmc-step", action="store_true",
                    help="run the headline form's first outer step once, eagerly, after the "
                         "copy probe, and exit (for rocprofv3 --pmc counter runs)")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write profiles/traffic.json from two rocprofv3 --pmc outputs and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU only: --gpus must be 1 (cells are independent, so a "
                                   "larger domain shards as contiguous cell ranges, one context "
                                   "per GPU, with no communication during integration)"}))
        sys.exit(2)
    # per-mechanism launches: with the 53-species inverse partly in registers
    # that launch holds 8 waves per CU, which the one-launch form (whose
    # 9-species cells share the 53-species register budget) cannot match
    workload, form = "mixed_s9_s53_1m", "batched"
    if args.traffic_from:
        print(json.dumps(traffic_from(*args.traffic_from, args.copy_probe, workload, form)))
        return
    w = W.make_workload(workload, args.cells)
    if args.copy_probe > 0:
        import torch
        n = int(args.copy_probe * 2**20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.pmc_step:
        import torch
        from paper_2405_01713_amd import bdfx
        integ = bdfx.Integrator(w["mechs"], w["y0"], w["rtol"], w["atol"], T=w["T"],
                                cell_mech=w["cell_mech"], **FORM_OPTS[form])
        integ.autotune(0.0, w["t_out"], cache=args.tuning_cache)
        y0 = integ.y.clone()
        if args.copy_probe > 0:  # the probe must precede the measured launches
            src = torch.ones(int(args.copy_probe * 2**20) // 8, dtype=torch.float64, device="cuda")
            torch.empty_like(src).copy_(src)
        integ.y.copy_(y0)
        integ.perturb(3, 0, w["perturb"])
        integ.integrate(0.0, w["t_out"])
        torch.cuda.synchronize()
        integ.close()
        log("pmc step done")
        return

    head = run_outer_loop(w, form, args.steps, args.warmup, tuning_cache=args.tuning_cache)
    log(f"headline {form}: {head['ms_per_outer_step']:.1f} ms per outer step")
    y_head = head.pop("_y")
    forms = {form: head}
    if not args.no_forms:
        for f in ("batched_fused", "batched_fp32lu", "plain"):
            r = run_outer_loop(w, f, w["outer_steps"], 0, tuning_cache=args.tuning_cache,
                               account=False)
            r["_y_sample"] = r.pop("_y")
            forms[f] = r
            log(f"headline workload {f}: {r['ms_per_outer_step']:.1f} ms per outer step")

    cpu = None
    if not args.no_cpu:
        c = cpu_baseline(w, args.cpu_sample)
        log(f"cpu baseline: {c['value']:.0f} cells/s on {c['cores']} threads")
        idx, yo = c.pop("_idx"), c.pop("_y")
        head["vs_oracle"] = dict(parity_summary(y_head[idx], yo, w["rtol"], w["atol"]),
                                 cells=int(idx.size))
        for f, r in forms.items():
            if f != form:
                r["vs_oracle"] = dict(parity_summary(r.pop("_y_sample")[idx], yo, w["rtol"],
                                                     w["atol"]), cells=int(idx.size))
        cpu = c
    for r in forms.values():
        r.pop("_y_sample", None)

    t_step = head["ms_per_outer_step"] * 1e-3
    F64, F32 = head["alg_flops_fp64_per_outer_step"], head["alg_flops_fp32_per_outer_step"]
    frac = roofline_frac(F64, F32, t_step)
    roof = {"bound": "alu", "achieved": frac * FP64_VECTOR_PEAK_TFLOPS,
            "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": frac,
            "traffic": stored_traffic(workload, form),
            "kernel": "bdfx::k_integrate (the 53- and the 9-species launch of each outer step)",
            "launches_per_outer_step": (1 if head.get("tuning") and all(
                t.get("fused") for t in head["tuning"]) else len(head.get("tuning") or w["mechs"])),
            "launch_ms": head.get("eager_integrate_ms_mean"),
            "flops_per_outer_step": F64 + F32,
            "alg_bytes_per_outer_step": int(sum(
                (16 * int(w["mechs"][k]["n_species"]) + 56) * int(np.sum(w["cell_mech"] == k))
                for k in range(len(w["mechs"]))))}
    extra = {}
    if not args.no_c1:
        extra["s21_r84_262k"] = run_c1(3, 1, tuning_cache=args.tuning_cache)
    if not args.no_adjoint:
        extra["adjoint"] = run_adjoint(3, 1)
    if not args.no_precision:
        extra["s53_r325_262k_fp32lu"] = run_precision(3, 1, tuning_cache=args.tuning_cache)
        extra["s53_r325_1m"] = run_precision(1, 1, tuning_cache=args.tuning_cache,
                                             n_cells=1 << 20)
    for name, fn in (("typical", run_typical), ("thermal", run_thermal), ("dq", run_dq),
                     ("gmres", run_gmres), ("lockstep", run_lockstep)):
        if name in args.extra.split(","):
            extra[name] = fn(tuning_cache=args.tuning_cache)
    parity = head.get("vs_oracle", {}).get("parity_ok")
    out = {
        "metric": "cells integrated/s per outer step @rtol 1e-6",
        "value": head["cells_per_s"],
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_outer_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": workload, "n_cells": w["n_cells"],
                   "species": [m["n_species"] for m in w["mechs"]],
                   "reactions": [m["n_reactions"] for m in w["mechs"]],
                   "outer_steps_per_graph": w["outer_steps"], "dt": w["t_out"],
                   "perturbation": w["perturb"], "rtol": w["rtol"], "atol": w["atol"],
                   "form": form},
        "parity_ok": parity,
        "roofline": roof,
        "cpu_baseline": cpu,
        "forms": forms,
        **extra,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
