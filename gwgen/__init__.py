"""Seeded synthetic inputs shaped like the paper's water-cluster workloads.

This module only draws random numbers and lays them out; it contains none of
the GW arithmetic, so both the FP64 oracle and the HIP path may consume it.

Shapes follow the paper's parallel-performance study (Section "Parallel
performance": water clusters, def2-QZVP / def2-universal-jkfit), which cannot
be reproduced here: there is no DFT, basis or geometry.  Every cluster of k
water molecules is stood in for by

  * n_occ = 5k, n_virt = 38k, N_aux = 112k;
  * occupied levels: k core levels at -20.5 Ha (jitter N(0, 0.01), i.e.
    standard deviation 0.1 Ha) and 4k valence levels uniform in
    [-1.3, -0.4] Ha; virtual levels uniform in [0.03, 5.0] Ha.  The monomer
    recipe is special: one core at exactly -20.5 Ha, four valence levels in
    [-1.3, -0.45] Ha and virtual levels in [0.05, 4.0] Ha;
  * orthonormalised three-index integrals B^P_pq (the tensor R = L^-1 E of
    Algorithm 1's initialisation) symmetric in p, q, drawn i.i.d. from
    N(0, 0.25 / (n_occ * n_virt)) for p <= q and mirrored.

Random streams are numpy's Philox4x64 counter-based generator keyed by
(seed, stream): stream 0 draws the levels, stream 1 + P draws the upper
triangle of B^P row-major.  Only B_ov (the occupied-virtual block) and the
rows B_nm of the requested states are kept, so the full B (44.7 GB for the
(H2O)30 shape) is never held in memory.

Layouts (row-major, float64):
  eps     [n_mo]                      ascending
  B_ov    [N_aux][n_occ * n_virt]     element (P, i*n_virt + a)
  B_rows  [n_rows][n_mo][N_aux]       element (r, m, P) = B^P_{row_ids[r], m}
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence

import numpy as np

__all__ = [
    "Shape", "Inputs", "CONFIGS", "cluster_shape", "monomer_shape",
    "make_eps", "make_inputs", "make_config", "serving_stream", "InputsUHF",
    "make_inputs_uhf",
]

# Sizes per water molecule (n_occ, n_virt, N_aux)
_PER_WATER = (5, 38, 112)


@dataclasses.dataclass(frozen=True)
class Shape:
    """Sizes and level recipe of one synthetic molecule."""
    n_occ: int
    n_virt: int
    n_aux: int
    n_core: int
    core_center: float = -20.5
    core_std: float = 0.1          # N(0, 0.01): variance 0.01
    valence: tuple = (-1.3, -0.4)
    virtual: tuple = (0.03, 5.0)

    @property
    def n_mo(self) -> int:
        return self.n_occ + self.n_virt

    @property
    def n_ov(self) -> int:
        return self.n_occ * self.n_virt


@dataclasses.dataclass
class Inputs:
    shape: Shape
    seed: int
    eps: np.ndarray          # [n_mo]
    B_ov: np.ndarray         # [N_aux][n_ov]
    row_ids: np.ndarray      # [n_rows] int32
    B_rows: np.ndarray       # [n_rows][n_mo][N_aux]

    @property
    def n_occ(self) -> int:
        return self.shape.n_occ


def monomer_shape() -> Shape:
    """Water monomer: exactly one core level (no jitter)."""
    return Shape(n_occ=5, n_virt=38, n_aux=112, n_core=1, core_std=0.0,
                 valence=(-1.3, -0.45), virtual=(0.05, 4.0))


def cluster_shape(k: int) -> Shape:
    """(H2O)_k-shaped cluster, k >= 1 (k = 1 uses the cluster recipe)."""
    if k < 1:
        raise ValueError("k must be >= 1")
    o, v, a = _PER_WATER
    return Shape(n_occ=o * k, n_virt=v * k, n_aux=a * k, n_core=k)


def custom_shape(n_occ: int, n_virt: int, n_aux: int, n_core: int = 1,
                 **kw) -> Shape:
    """Arbitrary sizes with the cluster level recipe (tests use ragged sizes)."""
    if not (0 <= n_core <= n_occ and n_occ >= 1 and n_virt >= 1 and n_aux >= 1):
        raise ValueError("bad shape")
    return Shape(n_occ=n_occ, n_virt=n_virt, n_aux=n_aux, n_core=n_core, **kw)


def _rng(seed: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(key=np.array([seed, stream], dtype=np.uint64)))


def make_eps(shape: Shape, seed: int) -> np.ndarray:
    """Ascending levels: cores, then valence, then virtual (each block sorted)."""
    r = _rng(seed, 0)
    core = shape.core_center + shape.core_std * r.standard_normal(shape.n_core)
    val = r.uniform(shape.valence[0], shape.valence[1], shape.n_occ - shape.n_core)
    vir = r.uniform(shape.virtual[0], shape.virtual[1], shape.n_virt)
    eps = np.concatenate([np.sort(core), np.sort(val), np.sort(vir)])
    if np.any(np.diff(eps) <= 0):
        raise RuntimeError("generated levels are not strictly ascending")
    return eps.astype(np.float64)


def make_inputs(shape: Shape, seed: int, row_ids: Sequence[int],
                b_scale: float = 1.0) -> Inputs:
    """Draw eps, B_ov and the requested rows B_nm.

    b_scale multiplies the standard deviation of B (1.0 = the recipe; 0.0
    gives the non-interacting limit used by edge-case tests).
    """
    n_occ, n_virt, n_aux, n_mo = shape.n_occ, shape.n_virt, shape.n_aux, shape.n_mo
    rows = np.asarray(list(row_ids), dtype=np.int32)
    if rows.size and (rows.min() < 0 or rows.max() >= n_mo):
        raise ValueError("row id out of range")
    eps = make_eps(shape, seed)
    std = b_scale * np.sqrt(0.25 / (n_occ * n_virt))
    n_tri = n_mo * (n_mo + 1) // 2
    # offset of row p inside the packed upper triangle (row-major, q >= p)
    p_idx = np.arange(n_mo)
    row_off = p_idx * n_mo - p_idx * (p_idx - 1) // 2
    occ = np.arange(n_occ)
    vir = np.arange(n_occ, n_mo)
    ov_idx = (row_off[occ][:, None] + (vir[None, :] - occ[:, None])).reshape(-1)
    # packed index of (min(n, m), max(n, m)) for each requested row n and every m
    m = np.arange(n_mo)
    if rows.size:
        lo = np.minimum(rows[:, None], m[None, :])
        hi = np.maximum(rows[:, None], m[None, :])
        row_idx = row_off[lo] + (hi - lo)
    else:
        row_idx = np.zeros((0, n_mo), dtype=np.int64)
    B_ov = np.empty((n_aux, n_occ * n_virt), dtype=np.float64)
    B_rows = np.empty((rows.size, n_mo, n_aux), dtype=np.float64)
    for P in range(n_aux):
        tri = _rng(seed, 1 + P).standard_normal(n_tri) * std
        B_ov[P] = tri[ov_idx]
        B_rows[:, :, P] = tri[row_idx]
    return Inputs(shape=shape, seed=seed, eps=eps, B_ov=B_ov, row_ids=rows, B_rows=B_rows)


def make_inputs_blocked(shape: Shape, seed: int, row_ids: Sequence[int]) -> Inputs:
    """Same distribution as make_inputs (symmetric B, i.i.d. N(0, 0.25/(n_occ n_virt))
    for p <= q), drawn block-wise so that large clusters are cheap: stream
    (seed, 1) draws B_ov [N_aux][n_ov] in one go, and stream (seed, 2 + r)
    draws, for requested row n = row_ids[r], the entries (n, m) that are not
    occupied-virtual pairs and have m >= n or m not requested; the remaining
    entries are copied from B_ov or from the mirror row, so B stays symmetric.
    Used for the serving workload (values differ from make_inputs)."""
    n_occ, n_virt, n_aux, n_mo = shape.n_occ, shape.n_virt, shape.n_aux, shape.n_mo
    rows = np.asarray(list(row_ids), dtype=np.int32)
    eps = make_eps(shape, seed)
    std = np.sqrt(0.25 / (n_occ * n_virt))
    B_ov = _rng(seed, 1).standard_normal((n_aux, n_occ * n_virt)) * std
    Bv = B_ov.reshape(n_aux, n_occ, n_virt)
    B_rows = np.empty((rows.size, n_mo, n_aux))
    pos = {int(n): r for r, n in enumerate(rows)}
    for r, n in enumerate(rows):
        n = int(n)
        own = _rng(seed, 2 + r).standard_normal((n_mo, n_aux)) * std
        for m in range(n_mo):
            if (n < n_occ) != (m < n_occ):           # occupied-virtual pair: from B_ov
                i, a = (n, m - n_occ) if n < n_occ else (m, n - n_occ)
                B_rows[r, m] = Bv[:, i, a]
            elif m in pos and m < n:                  # mirror of an earlier requested row
                B_rows[r, m] = B_rows[pos[m], n]
            else:
                B_rows[r, m] = own[m]
    return Inputs(shape=shape, seed=seed, eps=eps, B_ov=B_ov, row_ids=rows, B_rows=B_rows)


def full_B(inp_shape: Shape, seed: int, b_scale: float = 1.0) -> np.ndarray:
    """Full symmetric B [N_aux][n_mo][n_mo] (small shapes only)."""
    n_mo = inp_shape.n_mo
    if inp_shape.n_aux * n_mo * n_mo > 5e7:
        raise ValueError("full B requested for a large shape")
    std = b_scale * np.sqrt(0.25 / (inp_shape.n_occ * inp_shape.n_virt))
    n_tri = n_mo * (n_mo + 1) // 2
    iu = np.triu_indices(n_mo)
    B = np.zeros((inp_shape.n_aux, n_mo, n_mo))
    for P in range(inp_shape.n_aux):
        tri = _rng(seed, 1 + P).standard_normal(n_tri) * std
        B[P][iu] = tri
        B[P] = B[P] + np.triu(B[P], 1).T
    return B


@dataclasses.dataclass
class InputsUHF:
    """Open-shell inputs: one set of levels and integrals per spin (0 = up,
    1 = down) over a shared auxiliary basis.  States are named by their
    spin-orbital index sigma * n_mo + n."""
    n_mo: int
    n_occ: tuple            # (n_occ_up, n_occ_down)
    n_aux: int
    seed: int
    eps: np.ndarray         # [2][n_mo], each row ascending
    B_ov: tuple             # per spin [N_aux][n_occ_s * (n_mo - n_occ_s)]
    row_ids: np.ndarray     # [n_rows] int32 spin-orbital indices
    B_rows: np.ndarray      # [n_rows][n_mo][N_aux]: (P|n m) within the row's spin


def make_inputs_uhf(shape: Shape, seed: int, row_ids: Sequence[int], n_unpaired: int = 1,
                    same_spins: bool = False) -> InputsUHF:
    """Open-shell stand-in built from a closed-shell recipe: spin down has
    shape.n_occ occupied levels, spin up n_unpaired more (and as many fewer
    virtual).  Each spin draws its levels and its symmetric B from the recipe
    with its own key: spin up uses `seed`, spin down `seed + 2**32`.  With
    same_spins both spins take spin up's draws and n_unpaired must be 0 (the
    closed-shell inputs of make_inputs, twice)."""
    if same_spins and n_unpaired != 0:
        raise ValueError("same_spins needs n_unpaired = 0")
    n_mo = shape.n_mo
    occ = (shape.n_occ + n_unpaired, shape.n_occ)
    if not (1 <= occ[1] and occ[0] < n_mo):
        raise ValueError("bad open-shell occupation")
    rows = np.asarray(list(row_ids), dtype=np.int32)
    if rows.size and (rows.min() < 0 or rows.max() >= 2 * n_mo):
        raise ValueError("row id out of range")
    eps = np.empty((2, n_mo))
    B_ov = [None, None]
    B_rows = np.empty((rows.size, n_mo, shape.n_aux))
    for s in (0, 1):
        sh = dataclasses.replace(shape, n_occ=occ[s], n_virt=n_mo - occ[s])
        mine = [k for k, r in enumerate(rows) if r // n_mo == s]
        sub = make_inputs(sh, seed if (s == 0 or same_spins) else seed + (1 << 32),
                          [int(rows[k]) % n_mo for k in mine])
        eps[s] = sub.eps
        B_ov[s] = sub.B_ov
        for j, k in enumerate(mine):
            B_rows[k] = sub.B_rows[j]
    return InputsUHF(n_mo=n_mo, n_occ=occ, n_aux=shape.n_aux, seed=seed, eps=eps,
                     B_ov=tuple(B_ov), row_ids=rows, B_rows=B_rows)


# ---------------------------------------------------------------------------
# The five workloads (sizes, seeds and requested states)

@dataclasses.dataclass(frozen=True)
class Config:
    name: str
    shape: Shape
    seed: int
    grid_points: int
    states: tuple


def _homo_lumo_window(shape: Shape, below: int, above: int) -> tuple:
    homo = shape.n_occ - 1
    return tuple(range(homo - below, homo + 1 + 1 + above))


def _configs() -> dict:
    mono = monomer_shape()
    c2, c3, c4 = cluster_shape(10), cluster_shape(30), cluster_shape(20)
    return {
        "monomer": Config("monomer", mono, 1, 64, (mono.n_occ - 1, mono.n_occ)),
        "h2o10": Config("h2o10", c2, 2, 64, _homo_lumo_window(c2, 4, 4)),
        "h2o30": Config("h2o30", c3, 3, 128, _homo_lumo_window(c3, 9, 9)),
        "h2o20_core": Config("h2o20_core", c4, 4, 64, (0,)),
    }


CONFIGS = _configs()


def make_config(name: str, states: Optional[Sequence[int]] = None) -> Inputs:
    cfg = CONFIGS[name]
    return make_inputs(cfg.shape, cfg.seed, cfg.states if states is None else states)


def serving_stream(n_requests: int = 512, k_max: int = 24, seed: int = 5000,
                   rate: float = 1.0) -> List[dict]:
    """Request list for the serving workload: cluster size k ~ U{1..k_max},
    Poisson arrivals at `rate` requests per second, request r seeded 1000 + r,
    asking for HOMO-2..LUMO+2."""
    r = _rng(seed, 0)
    ks = r.integers(1, k_max + 1, size=n_requests)
    gaps = r.exponential(1.0 / rate, size=n_requests)
    t = np.cumsum(gaps) - gaps[0]
    out = []
    for i in range(n_requests):
        shape = cluster_shape(int(ks[i]))
        out.append({"id": i, "k": int(ks[i]), "seed": 1000 + i, "arrival_s": float(t[i]),
                    "shape": shape, "states": _homo_lumo_window(shape, 2, 2)})
    return out


def serving_inputs(k: int, seed: int) -> Inputs:
    """Inputs of one serving request: a (H2O)_k cluster asking for HOMO-2..LUMO+2."""
    shape = cluster_shape(k)
    return make_inputs_blocked(shape, seed, _homo_lumo_window(shape, 2, 2))
