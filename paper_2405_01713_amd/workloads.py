"""Seeded synthetic inputs for the batched stiff-kinetics integrator.

This module only *draws* inputs: mechanisms (species weights, reaction
stoichiometry, Arrhenius parameters, equilibrium constants) and per-cell
initial states, temperatures and rate-constant scalings.  It holds none of the
integration arithmetic (no rates, right-hand sides, Jacobians, norms or step
control), so that both the GPU path and the FP64 CPU oracle can consume the
same inputs without sharing any of the method.

The paper's production workloads (Pele's DRM21 / DOD53 / HEP88 mechanisms and
the Nyx cosmology states) are not available; these generators stand in for
them with the paper's species counts (21, 53), its largest batch of 64^3 cells
and mass-action kinetics (the chemistry source term R of the operator-split
system, Sec. 3.1, Eq. (7)).

Conventions
-----------
* State is molar concentration at unit density, ``y_i = Y_i / w_i``, laid out
  cell-major ``[N, S]`` (the paper's CY ordering, Sec. 4.1.2).
* A mechanism is a dict with int32 ``reac``/``prod`` ``[R, 3]`` species slots
  (``-1`` = empty, repeated species = stoichiometry), float64 ``lnA``,
  ``EaR`` (activation temperature, K) and ``lnK`` (natural log of the
  equilibrium constant, or ``None`` for irreversible reactions) and float64
  species weights ``w``.
"""
from __future__ import annotations

import numpy as np

SLOTS = 3

# Seeds used by the named workloads.
SEED_MECH = 1
SEED_STATE = 2
SEED_PERTURB = 3
SEED_LOSS = 4


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _slots(rows):
    out = np.full((len(rows), SLOTS), -1, dtype=np.int32)
    for r, sp in enumerate(rows):
        out[r, : len(sp)] = sp
    return out


def robertson_mechanism() -> dict:
    """Robertson's three-species stiff kinetics as three mass-action reactions.

    A -> B (k1 = 0.04), B + B -> B + C (k2 = 3e7), B + C -> A + C (k3 = 1e4).
    Isothermal (zero activation temperature), irreversible.
    """
    reac = _slots([[0], [1, 1], [1, 2]])
    prod = _slots([[1], [1, 2], [0, 2]])
    k = np.array([0.04, 3.0e7, 1.0e4])
    return dict(
        name="robertson",
        n_species=3,
        n_reactions=3,
        reac=reac,
        prod=prod,
        lnA=np.log(k),
        EaR=np.zeros(3),
        lnK=None,
        w=np.ones(3),
    )


def synthetic_mechanism(n_species: int, n_reactions: int, seed: int = SEED_MECH) -> dict:
    """Reversible association reactions A + B <=> C with w_C = w_A + w_B.

    Species ``i`` has integer weight ``i + 1``.  Triples ``(a <= b, c = a + b)``
    are drawn without replacement while the pool lasts and with replacement
    afterwards (duplicates get their own Arrhenius draws).  ``log10 A ~
    U[8, 14]``, ``Ea/R ~ U[0, 3e4]`` K, and reverse rates follow detailed
    balance with species potentials ``g_i ~ U[0, 5]``:
    ``ln K_r = g_A + g_B - g_C``.
    """
    S, R = int(n_species), int(n_reactions)
    rng = _rng(seed)
    pool = [(a, b, a + b) for c in range(2, S + 1) for a in range(1, c // 2 + 1) for b in (c - a,)]
    pool = [t for t in pool if t[0] <= t[1]]
    if not pool:
        raise ValueError("need at least two species for association reactions")
    pool_arr = np.array(pool, dtype=np.int64)
    n_unique = min(R, len(pool))
    pick = list(rng.permutation(len(pool))[:n_unique])
    if R > n_unique:
        pick += list(rng.integers(0, len(pool), size=R - n_unique))
    trip = pool_arr[np.array(pick, dtype=np.int64)] - 1  # species index = weight - 1
    log10A = rng.uniform(8.0, 14.0, size=R)
    EaR = rng.uniform(0.0, 3.0e4, size=R)
    g = rng.uniform(0.0, 5.0, size=S)
    reac = np.full((R, SLOTS), -1, dtype=np.int32)
    prod = np.full((R, SLOTS), -1, dtype=np.int32)
    reac[:, 0] = trip[:, 0]
    reac[:, 1] = trip[:, 1]
    prod[:, 0] = trip[:, 2]
    lnK = g[trip[:, 0]] + g[trip[:, 1]] - g[trip[:, 2]]
    return dict(
        name=f"synthetic_s{S}_r{R}",
        n_species=S,
        n_reactions=R,
        reac=reac,
        prod=prod,
        lnA=log10A * np.log(10.0),
        EaR=EaR,
        lnK=lnK,
        w=np.arange(1, S + 1, dtype=np.float64),
        g=g,
    )


def thermal_mechanism(mech: dict, seed: int = 17) -> dict:
    """The mechanism with synthetic thermochemistry for a non-isothermal
    cell: heat capacity ``cv_i = 1.5 + 0.5 w_i`` and energy at zero
    temperature ``u0_i = 1000 w_i + d_i`` with ``d_i ~ U[-300, 300]`` (the
    weight-proportional part cancels in every A + B <=> C reaction, so
    reaction energies come from ``d`` and from the heat-capacity change)."""
    rng = _rng(seed)
    w = np.asarray(mech["w"], dtype=np.float64)
    d = rng.uniform(-300.0, 300.0, size=w.size)
    return dict(mech, name=mech.get("name", "mech") + "_thermal", cv=1.5 + 0.5 * w,
                u0=1000.0 * w + d)


def unimolecular_mechanism(n_species: int, n_reactions: int, seed: int) -> dict:
    """Random first-order network (A -> B), i.e. a linear system y' = K y."""
    S, R = int(n_species), int(n_reactions)
    rng = _rng(seed)
    reac = np.full((R, SLOTS), -1, dtype=np.int32)
    prod = np.full((R, SLOTS), -1, dtype=np.int32)
    for r in range(R):
        a, b = rng.choice(S, size=2, replace=False)
        reac[r, 0], prod[r, 0] = a, b
    return dict(
        name=f"unimolecular_s{S}_r{R}",
        n_species=S,
        n_reactions=R,
        reac=reac,
        prod=prod,
        lnA=rng.uniform(-1.0, 3.0, size=R) * np.log(10.0),
        EaR=np.zeros(R),
        lnK=None,
        w=np.ones(S),
    )


def cell_states(mech: dict, n_cells: int, seed: int = SEED_STATE,
                T_range=(1000.0, 2500.0)) -> dict:
    """Per-cell temperature ``T ~ U[T_range]`` and mass fractions Dirichlet(1)."""
    S = mech["n_species"]
    rng = _rng(seed)
    T = rng.uniform(T_range[0], T_range[1], size=n_cells)
    Y = rng.dirichlet(np.ones(S), size=n_cells)
    y = Y / mech["w"][None, :]
    return dict(y0=np.ascontiguousarray(y), T=T)


def robertson_cells(n_cells: int, seed: int = SEED_STATE, sigma: float = 0.1) -> dict:
    """Robertson cells: y0 = (1, 0, 0), each k scaled by lognormal(sigma)."""
    rng = _rng(seed)
    kscale = np.exp(sigma * rng.standard_normal(size=(n_cells, 3)))
    y0 = np.zeros((n_cells, 3))
    y0[:, 0] = 1.0
    return dict(y0=y0, kscale=kscale, T=None)


def mixed_cells(mechs, n_cells: int, seed: int = SEED_STATE,
                T_range=(800.0, 2800.0)) -> dict:
    """Cells split at random (equal probability) between ``mechs``.

    Returns ``cell_mech`` (int32 ``[N]``) and ``y0`` padded to ``S_max``
    columns with zeros beyond each cell's own species count.
    """
    rng = _rng(seed)
    n_mech = len(mechs)
    cell_mech = rng.integers(0, n_mech, size=n_cells).astype(np.int32)
    T = rng.uniform(T_range[0], T_range[1], size=n_cells)
    S_max = max(m["n_species"] for m in mechs)
    y0 = np.zeros((n_cells, S_max))
    for k, m in enumerate(mechs):
        idx = np.nonzero(cell_mech == k)[0]
        S = m["n_species"]
        Y = rng.dirichlet(np.ones(S), size=idx.size)
        y0[idx, :S] = Y / m["w"][None, :]
    return dict(y0=y0, T=T, cell_mech=cell_mech)


def loss_weights(n_species: int, seed: int = SEED_LOSS) -> np.ndarray:
    """Loss weights ``c ~ N(0, 1)`` shared by all cells."""
    return _rng(seed).standard_normal(size=n_species)


# ---------------------------------------------------------------------------
# Named workloads (sizes of the benchmark configurations)
# ---------------------------------------------------------------------------

WORKLOADS = {
    "robertson_4k": dict(kind="robertson", n_cells=4096, t_out=40.0, rtol=1e-6, atol=1e-10),
    "s21_r84_262k": dict(kind="synthetic", S=21, R=84, n_cells=262144, t_out=1e-5,
                         rtol=1e-6, atol=1e-10, T_range=(1000.0, 2500.0)),
    "mixed_s9_s53_1m": dict(kind="mixed", mechs=((9, 30), (53, 325)), n_cells=1048576,
                            t_out=1e-5, outer_steps=10, perturb=0.01, rtol=1e-6, atol=1e-10,
                            T_range=(800.0, 2800.0)),
    "s53_r325_262k_fp32lu": dict(kind="synthetic53", S=53, R=325, n_cells=262144, t_out=1e-5,
                                 rtol=1e-6, atol=1e-10, T_range=(1000.0, 2500.0)),
    "s21_r84_65k_adjoint": dict(kind="synthetic", S=21, R=84, n_cells=65536, t_out=1e-5,
                                rtol=1e-6, atol=1e-10, T_range=(1000.0, 2500.0), state_seed=5),
    # non-isothermal: temperature is the state's last component (atol 1e-6 K)
    "s21_r84_thermal_262k": dict(kind="thermal", S=21, R=84, n_cells=262144, t_out=1e-5,
                                 rtol=1e-6, atol=1e-10, atol_T=1e-6, T_range=(1000.0, 2500.0)),
}

# Mechanism seeds: the mixed workload draws its two mechanisms from seeds 1 and
# 11; the 53-species precision workload reuses the mixed workload's 53/325
# mechanism.
MECH_SEED_S9 = 1
MECH_SEED_S53 = 11


def make_workload(name: str, n_cells: int | None = None) -> dict:
    """Materialise a named workload (optionally with fewer cells)."""
    spec = dict(WORKLOADS[name])
    N = int(n_cells if n_cells is not None else spec["n_cells"])
    out = dict(name=name, rtol=spec["rtol"], atol=spec["atol"], t0=0.0, t_out=spec["t_out"],
               n_cells=N, outer_steps=spec.get("outer_steps", 1), perturb=spec.get("perturb", 0.0))
    kind = spec["kind"]
    if kind == "robertson":
        m = robertson_mechanism()
        c = robertson_cells(N)
        out.update(mechs=[m], y0=c["y0"], kscale=c["kscale"], T=None, cell_mech=None)
    elif kind == "synthetic":
        m = synthetic_mechanism(spec["S"], spec["R"], SEED_MECH)
        c = cell_states(m, N, spec.get("state_seed", SEED_STATE), spec["T_range"])
        out.update(mechs=[m], y0=c["y0"], T=c["T"], kscale=None, cell_mech=None)
    elif kind == "synthetic53":
        m = synthetic_mechanism(spec["S"], spec["R"], MECH_SEED_S53)
        c = cell_states(m, N, SEED_STATE, spec["T_range"])
        out.update(mechs=[m], y0=c["y0"], T=c["T"], kscale=None, cell_mech=None)
    elif kind == "thermal":
        m0 = synthetic_mechanism(spec["S"], spec["R"], SEED_MECH)
        m = thermal_mechanism(m0)
        c = cell_states(m0, N, spec.get("state_seed", SEED_STATE), spec["T_range"])
        y0 = np.concatenate([c["y0"], c["T"][:, None]], axis=1)
        out.update(mechs=[m], y0=y0, T=None, kscale=None, cell_mech=None,
                   atol=np.array([spec["atol"]] * spec["S"] + [spec["atol_T"]]))
    elif kind == "mixed":
        (s1, r1), (s2, r2) = spec["mechs"]
        ms = [synthetic_mechanism(s1, r1, MECH_SEED_S9), synthetic_mechanism(s2, r2, MECH_SEED_S53)]
        c = mixed_cells(ms, N, SEED_STATE, spec["T_range"])
        out.update(mechs=ms, y0=c["y0"], T=c["T"], kscale=None, cell_mech=c["cell_mech"])
    else:  # pragma: no cover
        raise KeyError(kind)
    return out
