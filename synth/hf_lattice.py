"""Seeded synthetic inputs shaped like the HF molecular crystal of the paper.

The paper's calculations (Sec. IV, HF crystal cubes up to 10x10x10 molecules,
32 orbitals per molecule with 5 doubly occupied) use real integrals that are
not available here.  This module draws inputs of the same shapes:

* monomers on a simple cubic lattice, 3.4 Angstrom spacing, open boundaries
  (the paper uses no periodic boundary conditions);
* per monomer: o occupied and v virtual orbital energies (Eh), occupied drawn
  from U[-1.5, -0.5], virtual from U[0.2, 3.0], and an intra-monomer block
  K[i, j, a, b] = <ab|ij> drawn N(0, 0.05^2) and antisymmetrised in (i, j) and
  in (a, b);
* per unordered pair inside the cutoff: a dimer block V[i, a, j, b] = (ai|bj)
  with i, a on the first monomer and j, b on the second, drawn
  N(0, 1) * 0.05 * (3.4 / R)^3 * coupling_scale.

Every value is keyed by a numpy SeedSequence built from the workload id, the
cluster id, the kind of draw and the integer lattice coordinates of the site(s)
involved, so inputs do not depend on monomer numbering or generation order.

This module holds none of the method's arithmetic: it only draws numbers and
builds the lattice and the cutoff pair list.
"""
from __future__ import annotations

import contextlib
import dataclasses
import math
import threading

import numpy as np

SEED_ROOT = 14092700
SPACING_A = 3.4
SIGMA_K = 0.05
SIGMA_V = 0.05
EPS_OCC = (-1.5, -0.5)
EPS_VIR = (0.2, 3.0)
# default coupling scale: at scale 1 the sweep map of these random blocks has a
# dominant eigenvalue > 1 and Jacobi diverges.  The doubles sweep map depends on
# the couplings through 2 x scale^2 (spin-summed pair term times V twice), and
# 0.18 puts the 1000-monomer crystal at about the 15 micro-iterations the paper
# reports; the singles map (linear in the scale) then contracts by about 0.6
DEFAULT_COUPLING_SCALE = 0.18

KIND_MONOMER = 0
KIND_PAIR = 1
KIND_CLUSTER = 2
KIND_STREAM = 3
KIND_SINGLES = 4
SIGMA_W = 0.05
KIND_LCCD = 5
SIGMA_LCCD = 0.01
# the full monomer equation's ring terms contract K with the amplitudes; at the
# stated sigma 0.05 of K the sweep map of random blocks has a dominant eigenvalue
# > 1, so workloads with the intramonomer terms draw K at 0.2 x 0.05 = 0.01
LCCD_K_SCALE = 0.2


@dataclasses.dataclass
class Problem:
    """Flat, concatenated MCPT(2) inputs (the layout the C-ABI takes).

    eps:   concatenated per monomer, o_X occupied then v_X virtual energies
    k:     concatenated K_X[i][j][a][b] = <ab|ij>, row-major (o, o, v, v)
    pairs: [P, 2] monomer indices (X, Y), X != Y, each unordered pair once
    v:     concatenated V_XY[i][a][j][b] = (ai|bj), row-major (oX, vX, oY, vY)
    """
    n_occ: np.ndarray
    n_vir: np.ndarray
    eps: np.ndarray
    k: np.ndarray
    pairs: np.ndarray
    v: np.ndarray
    sites: np.ndarray | None = None
    meta: dict = dataclasses.field(default_factory=dict)

    def __post_init__(self):
        self.n_occ = np.ascontiguousarray(self.n_occ, dtype=np.int32)
        self.n_vir = np.ascontiguousarray(self.n_vir, dtype=np.int32)
        self.pairs = np.ascontiguousarray(np.asarray(self.pairs, dtype=np.int32).reshape(-1, 2))
        o = self.n_occ.astype(np.int64)
        v = self.n_vir.astype(np.int64)
        self.eps_off = np.concatenate([[0], np.cumsum(o + v)])
        self.k_off = np.concatenate([[0], np.cumsum(o * o * v * v)])
        nx = o * v
        if len(self.pairs):
            sizes = nx[self.pairs[:, 0]] * nx[self.pairs[:, 1]]
        else:
            sizes = np.zeros(0, dtype=np.int64)
        self.v_off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)

    # -- sizes ------------------------------------------------------------
    @property
    def n_mono(self) -> int:
        return int(len(self.n_occ))

    @property
    def n_pair(self) -> int:
        return int(len(self.pairs))

    def n_ov(self, x: int) -> int:
        return int(self.n_occ[x]) * int(self.n_vir[x])

    # -- views ------------------------------------------------------------
    def eps_of(self, x: int):
        o = int(self.n_occ[x])
        e = self.eps[self.eps_off[x]:self.eps_off[x + 1]]
        return e[:o], e[o:]

    def k_of(self, x: int) -> np.ndarray:
        o, v = int(self.n_occ[x]), int(self.n_vir[x])
        return self.k[self.k_off[x]:self.k_off[x + 1]].reshape(o, o, v, v)

    def v_of(self, p: int) -> np.ndarray:
        x, y = (int(t) for t in self.pairs[p])
        return self.v[self.v_off[p]:self.v_off[p + 1]].reshape(
            int(self.n_occ[x]), int(self.n_vir[x]), int(self.n_occ[y]), int(self.n_vir[y]))

    def nbytes(self) -> int:
        return int(self.eps.nbytes + self.k.nbytes + self.v.nbytes + self.pairs.nbytes)

    # -- transformations used by invariance tests ---------------------------
    def relabel(self, perm, flip=None) -> "Problem":
        """New problem with monomer old index perm[new] at position new; pairs
        whose flip flag is set are stored in the reverse orientation (V -> V^T
        over the (i,a) <-> (j,b) index pairs)."""
        perm = np.asarray(perm, dtype=np.int64)
        inv = np.empty_like(perm)
        inv[perm] = np.arange(len(perm))
        n_occ = self.n_occ[perm]
        n_vir = self.n_vir[perm]
        eps = np.concatenate([self.eps[self.eps_off[x]:self.eps_off[x + 1]] for x in perm]) \
            if len(perm) else np.zeros(0)
        k = np.concatenate([self.k[self.k_off[x]:self.k_off[x + 1]] for x in perm]) \
            if len(perm) else np.zeros(0)
        flip = np.zeros(self.n_pair, dtype=bool) if flip is None else np.asarray(flip, dtype=bool)
        pairs = []
        blocks = []
        for p in range(self.n_pair):
            x, y = (int(t) for t in self.pairs[p])
            vb = self.v_of(p)
            if flip[p]:
                pairs.append((inv[y], inv[x]))
                blocks.append(np.ascontiguousarray(vb.transpose(2, 3, 0, 1)).ravel())
            else:
                pairs.append((inv[x], inv[y]))
                blocks.append(vb.ravel())
        v = np.concatenate(blocks) if blocks else np.zeros(0)
        sites = self.sites[perm] if self.sites is not None else None
        return Problem(n_occ, n_vir, eps, k, np.array(pairs, dtype=np.int32).reshape(-1, 2), v,
                       sites, dict(self.meta, relabelled=True))

    def subset_pairs(self, keep) -> "Problem":
        keep = np.asarray(keep, dtype=bool)
        blocks = [self.v[self.v_off[p]:self.v_off[p + 1]] for p in range(self.n_pair) if keep[p]]
        v = np.concatenate(blocks) if blocks else np.zeros(0)
        return Problem(self.n_occ, self.n_vir, self.eps, self.k, self.pairs[keep], v,
                       self.sites, dict(self.meta))


def concat_problems(probs) -> Problem:
    """Disjoint union of clusters (no pairs between clusters)."""
    n_occ = np.concatenate([p.n_occ for p in probs])
    n_vir = np.concatenate([p.n_vir for p in probs])
    eps = np.concatenate([p.eps for p in probs])
    k = np.concatenate([p.k for p in probs])
    shift = np.concatenate([[0], np.cumsum([p.n_mono for p in probs])])
    pairs = np.concatenate([p.pairs.astype(np.int64) + shift[i] for i, p in enumerate(probs)]) \
        if probs else np.zeros((0, 2))
    v = np.concatenate([p.v for p in probs])
    return Problem(n_occ, n_vir, eps, k, pairs, v, None, {"union_of": len(probs)})


# ---------------------------------------------------------------------------
# lattice geometry
# ---------------------------------------------------------------------------
def cubic_sites(nx: int, ny: int, nz: int) -> np.ndarray:
    """Integer lattice coordinates of an nx x ny x nz block, lexicographic order."""
    g = np.stack(np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij"), -1)
    return g.reshape(-1, 3).astype(np.int64)


def cluster_sites(n: int) -> np.ndarray:
    """First n sites (lexicographic) of the smallest cube holding n sites."""
    side = 1
    while side ** 3 < n:
        side += 1
    return cubic_sites(side, side, side)[:n]


def pair_list(sites: np.ndarray, cutoff_spacings: float | None) -> np.ndarray:
    """All unordered pairs X < Y whose lattice distance is within the cutoff.

    The cutoff is inclusive and measured between lattice sites in units of the
    spacing; it is applied on squared integer distances, so it is exact.
    Open boundaries: no periodic images."""
    n = len(sites)
    if n < 2:
        return np.zeros((0, 2), dtype=np.int32)
    iu, ju = np.triu_indices(n, 1)
    d = sites[iu] - sites[ju]
    d2 = np.einsum("ij,ij->i", d, d)
    if cutoff_spacings is None:
        keep = np.ones(len(d2), dtype=bool)
    else:
        keep = d2 <= int(math.floor(cutoff_spacings ** 2 + 1e-9))
    return np.stack([iu[keep], ju[keep]], 1).astype(np.int32)


# ---------------------------------------------------------------------------
# seeded draws
# ---------------------------------------------------------------------------
def _rng(*key) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([SEED_ROOT, *[int(k) for k in key]]))


def _monomer_draw(workload: int, cluster: int, site, o: int | None, v: int | None,
                  mixed_sizes: bool = False):
    rng = _rng(workload, cluster, KIND_MONOMER, *site)
    # the size-class draw is always taken so the other draws do not depend on it
    u = rng.random()
    if mixed_sizes:
        o, v = (5, 27) if u < 0.5 else (8, 56)
    e_occ = np.sort(rng.uniform(*EPS_OCC, size=o))
    e_vir = np.sort(rng.uniform(*EPS_VIR, size=v))
    g = rng.normal(0.0, SIGMA_K, size=(o, o, v, v))
    # antisymmetrise in (i, j) and (a, b); keeps sigma = 0.05 off the zero diagonals
    k = 0.5 * (g - g.transpose(1, 0, 2, 3) - g.transpose(0, 1, 3, 2) + g.transpose(1, 0, 3, 2))
    return o, v, np.concatenate([e_occ, e_vir]), k


def _pair_block(workload: int, cluster: int, site_x, site_y, shape, r_angstrom: float,
                coupling_scale: float) -> np.ndarray:
    rng = _rng(workload, cluster, KIND_PAIR, *site_x, *site_y)
    z = rng.standard_normal(size=shape)
    return (coupling_scale * SIGMA_V * (SPACING_A / r_angstrom) ** 3) * z


def make_lattice_problem(sites: np.ndarray, cutoff_spacings: float | None, *, o: int = 5,
                         v: int = 27, workload: int = 0, cluster: int = 0,
                         coupling_scale: float = DEFAULT_COUPLING_SCALE,
                         mixed_sizes: bool = False, displacement=None,
                         dtype_v=np.float64, sizes=None, k_scale: float = 1.0) -> Problem:
    """Build a problem on the given integer lattice sites.

    displacement: None or (monomer index, axis 0..2, signed shift in Angstrom);
    the displaced monomer keeps its energies and intra block, its pair blocks
    are rescaled by (R0 / R)^3 and the pair list stays that of the undisplaced
    lattice (fixed topology).  sizes: optional per-monomer (o, v) list.
    k_scale multiplies every intra block (the same seeded draw, rescaled)."""
    sites = np.asarray(sites, dtype=np.int64)
    n = len(sites)
    n_occ = np.empty(n, dtype=np.int32)
    n_vir = np.empty(n, dtype=np.int32)
    eps_parts, k_parts = [], []
    for x in range(n):
        so, sv = (sizes[x] if sizes is not None else (o, v))
        ox, vx, e, k = _monomer_draw(workload, cluster, sites[x], so, sv, mixed_sizes)
        n_occ[x], n_vir[x] = ox, vx
        eps_parts.append(e)
        k_parts.append(k.ravel() * k_scale if k_scale != 1.0 else k.ravel())
    pairs = pair_list(sites, cutoff_spacings)
    pos = sites.astype(np.float64) * SPACING_A
    if displacement is not None:
        dx, axis, shift = displacement
        pos_new = pos.copy()
        pos_new[int(dx), int(axis)] += float(shift)
    else:
        pos_new = pos
    nxv = n_occ.astype(np.int64) * n_vir
    sizes = nxv[pairs[:, 0]] * nxv[pairs[:, 1]] if len(pairs) else np.zeros(0, dtype=np.int64)
    vflat = np.empty(int(sizes.sum()), dtype=dtype_v)
    off = 0
    for p, (x, y) in enumerate(pairs):
        shape = (int(n_occ[x]), int(n_vir[x]), int(n_occ[y]), int(n_vir[y]))
        r0 = float(np.linalg.norm(pos[x] - pos[y]))
        blk = _pair_block(workload, cluster, sites[x], sites[y], shape, r0, coupling_scale)
        if displacement is not None and (x == displacement[0] or y == displacement[0]):
            r1 = float(np.linalg.norm(pos_new[x] - pos_new[y]))
            blk *= (r0 / r1) ** 3
        sz = int(sizes[p])
        vflat[off:off + sz] = blk.ravel()
        off += sz
    eps = np.concatenate(eps_parts) if eps_parts else np.zeros(0)
    k = np.concatenate(k_parts) if k_parts else np.zeros(0)
    return Problem(n_occ, n_vir, eps, k, pairs, vflat, sites,
                   dict(workload=workload, cluster=cluster, cutoff=cutoff_spacings,
                        coupling_scale=coupling_scale, displacement=displacement, k_scale=k_scale))


# named workloads: the HF-crystal-shaped cubes (o=5, v=27, 32 orbitals/monomer)
WORKLOADS = {
    "hf-2x2x2": dict(workload=1, dims=(2, 2, 2), cutoff=None),
    "hf-5x5x5-c2": dict(workload=2, dims=(5, 5, 5), cutoff=2.0),
    "hf-10x10x10-c3": dict(workload=3, dims=(10, 10, 10), cutoff=3.0),
}


def make_workload(name: str, coupling_scale: float = DEFAULT_COUPLING_SCALE, **kw) -> Problem:
    spec = WORKLOADS[name]
    p = make_lattice_problem(cubic_sites(*spec["dims"]), spec["cutoff"], workload=spec["workload"],
                             coupling_scale=coupling_scale, **kw)
    p.meta["name"] = name
    return p


def cluster_batch_sizes(n_clusters: int = 64, *, workload: int = 4, min_mono: int = 27,
                        max_mono: int = 512, first: int = 0) -> list:
    """Monomer counts of the clusters make_cluster_batch draws (log-uniform)."""
    out = []
    for c in range(first, first + n_clusters):
        rng = _rng(workload, c, KIND_CLUSTER)
        out.append(int(round(math.exp(rng.uniform(math.log(min_mono), math.log(max_mono))))))
    return out


def make_cluster_batch(n_clusters: int = 64, *, workload: int = 4, min_mono: int = 27,
                       max_mono: int = 512, cutoff: float = 2.0,
                       coupling_scale: float = DEFAULT_COUPLING_SCALE, mixed_sizes: bool = True,
                       dtype_v=np.float64, first: int = 0, only=None, workers: int = 1):
    """Uneven cubic-lattice clusters: n_mono log-uniform in [min, max], each
    monomer o5v27 or o8v56 with probability 1/2.  only: optional list of cluster
    indices to make (the others are skipped).  workers > 1 draws clusters on
    that many threads (every draw is keyed by cluster and site, so the values
    do not depend on it; NumPy's generators release the GIL)."""
    sizes = cluster_batch_sizes(n_clusters, workload=workload, min_mono=min_mono, max_mono=max_mono,
                                first=first)
    which = [c for c in range(first, first + n_clusters) if only is None or c in only]

    def one(c):
        p = make_lattice_problem(cluster_sites(sizes[c - first]), cutoff, workload=workload, cluster=c,
                                 coupling_scale=coupling_scale, mixed_sizes=mixed_sizes,
                                 dtype_v=dtype_v)
        p.meta["name"] = f"cluster-{c}"
        return p

    if workers <= 1:
        return [one(c) for c in which]
    from concurrent.futures import ThreadPoolExecutor
    # largest clusters first so the pool drains evenly; results in cluster order
    order = sorted(which, key=lambda c: -sizes[c - first])
    with ThreadPoolExecutor(max_workers=workers) as ex:
        made = dict(zip(order, ex.map(one, order)))
    return [made[c] for c in which]


def make_served_request(r: int, *, workload: int = 5, min_mono: int = 8, max_mono: int = 1000,
                        cutoff: float = 3.0, step_angstrom: float = 0.01,
                        coupling_scale: float = DEFAULT_COUPLING_SCALE):
    """One served request: a cluster of log-uniform size with one monomer
    displaced by +-0.01 Angstrom along a seeded axis (finite-difference geometry,
    Sec. IV.A)."""
    rng = _rng(workload, r, KIND_STREAM)
    n = int(round(math.exp(rng.uniform(math.log(min_mono), math.log(max_mono)))))
    mono = int(rng.integers(0, n))
    axis = int(rng.integers(0, 3))
    sign = 1.0 if rng.random() < 0.5 else -1.0
    p = make_lattice_problem(cluster_sites(n), cutoff, workload=workload, cluster=r,
                             coupling_scale=coupling_scale,
                             displacement=(mono, axis, sign * step_angstrom))
    p.meta["name"] = f"request-{r}"
    return p


class ServedStream:
    """The served stream cut from one resident crystal `base`: request r is the
    n monomers nearest the crystal's centre (n log-uniform in [min_mono,
    max_mono]; distance ties by index), every pair of `base` between them with
    its block, and one of them displaced by +-step along a seeded axis (blocks of
    its pairs rescaled by (R0 / R)^3, pair list unchanged) - the finite-
    displacement geometries of the paper's frequency workflow.

    The crystal is relabelled once by distance from its centre, with its pairs
    ordered by their larger new index, so the monomers and pairs of every request
    are prefixes of the relabelled arrays: making a request is one slice copy of
    its blocks plus the rescaled blocks of the displaced monomer."""

    def __init__(self, base: Problem, *, workload: int = 5, min_mono: int = 8, max_mono: int | None = None,
                 step_angstrom: float = 0.01):
        self.workload, self.min_mono, self.step = workload, min_mono, step_angstrom
        N = base.n_mono
        self.max_mono = N if max_mono is None else min(max_mono, N)
        sites = np.asarray(base.sites, dtype=np.int64)
        d2 = ((sites - sites.mean(axis=0)) ** 2).sum(axis=1)
        order = np.lexsort((np.arange(N), d2))            # new index -> old index
        inv = np.empty(N, dtype=np.int64)
        inv[order] = np.arange(N)
        self.n_occ, self.n_vir = base.n_occ[order].copy(), base.n_vir[order].copy()
        self.sites = sites[order]
        self.eps = np.concatenate([base.eps[base.eps_off[x]:base.eps_off[x + 1]] for x in order])
        self.k = np.concatenate([base.k[base.k_off[x]:base.k_off[x + 1]] for x in order])
        self.eoff = np.concatenate([[0], np.cumsum(self.n_occ.astype(np.int64) + self.n_vir)])
        nxv = self.n_occ.astype(np.int64) * self.n_vir
        self.koff = np.concatenate([[0], np.cumsum(nxv * nxv)])
        px, py = inv[base.pairs[:, 0]], inv[base.pairs[:, 1]]
        hi = np.maximum(px, py)
        porder = np.lexsort((np.minimum(px, py), hi))
        self.pairs = np.stack([px[porder], py[porder]], axis=1).astype(np.int32)
        self.v = np.concatenate([base.v[base.v_off[p]:base.v_off[p + 1]] for p in porder])
        psz = nxv[self.pairs[:, 0]] * nxv[self.pairs[:, 1]]
        self.voff = np.concatenate([[0], np.cumsum(psz)])
        self.pairs_below = np.searchsorted(hi[porder], np.arange(N + 1), side="left")   # pairs among the first n
        self.meta = dict(base.meta)
        self._lock = threading.Lock()

    def draw(self, r: int):
        """(n, displaced monomer, axis, signed shift) of request r."""
        rng = _rng(self.workload, r, KIND_STREAM)
        n = int(round(math.exp(rng.uniform(math.log(self.min_mono), math.log(self.max_mono)))))
        n = max(1, min(n, self.max_mono))
        mono = int(rng.integers(0, n))
        axis = int(rng.integers(0, 3))
        sign = 1.0 if rng.random() < 0.5 else -1.0
        return n, mono, axis, sign * self.step

    def _scales(self, n, mono, axis, shift):
        """(pair index, factor) of the displaced monomer's pairs among the first n monomers."""
        P = int(self.pairs_below[n])
        pairs = self.pairs[:P]
        pos = self.sites[:n].astype(np.float64) * SPACING_A
        moved = pos[mono].copy()
        moved[axis] += shift
        out = []
        for p in np.flatnonzero((pairs[:, 0] == mono) | (pairs[:, 1] == mono)):
            x, y = int(pairs[p, 0]), int(pairs[p, 1])
            other = pos[y] if x == mono else pos[x]
            out.append((int(p), (float(np.linalg.norm(pos[mono] - other)) /
                                 float(np.linalg.norm(moved - other))) ** 3))
        return P, out

    def _problem(self, r, n, P, v, shift_info):
        meta = dict(self.meta)
        meta.update(name=f"served-{r}", displacement=shift_info, carved_from=len(self.n_occ))
        return Problem(self.n_occ[:n], self.n_vir[:n], self.eps[:self.eoff[n]], self.k[:self.koff[n]],
                       self.pairs[:P], v, self.sites[:n], meta)

    def request(self, r: int) -> Problem:
        """Request r as a problem of its own (its blocks copied)."""
        n, mono, axis, shift = self.draw(r)
        P, scales = self._scales(n, mono, axis, shift)
        v = self.v[:self.voff[P]].copy()
        for p, f in scales:
            v[self.voff[p]:self.voff[p + 1]] *= f
        return self._problem(r, n, P, v, (mono, axis, shift))

    @contextlib.contextmanager
    def lend(self, r: int):
        """Request r as views of the relabelled crystal, for a caller that copies
        it (an upload or submission) before the block ends: the displaced
        monomer's blocks are scaled in place and restored afterwards, one
        request at a time."""
        n, mono, axis, shift = self.draw(r)
        P, scales = self._scales(n, mono, axis, shift)
        with self._lock:
            saved = [(p, self.v[self.voff[p]:self.voff[p + 1]].copy()) for p, _ in scales]
            for p, f in scales:
                self.v[self.voff[p]:self.voff[p + 1]] *= f
            try:
                yield self._problem(r, n, P, self.v[:self.voff[P]], (mono, axis, shift))
            finally:
                for p, blk in saved:
                    self.v[self.voff[p]:self.voff[p + 1]] = blk


def carve_served_request(base: Problem, r: int, *, workload: int = 5, min_mono: int = 8,
                         max_mono: int | None = None, step_angstrom: float = 0.01) -> Problem:
    """Request r of a served stream carved out of a resident crystal `base`:
    the n monomers nearest the crystal's centre (n log-uniform in
    [min_mono, max_mono], ties by index), every pair of `base` between them with
    its block, and one of them displaced by +-step along a seeded axis (blocks
    of its pairs rescaled by (R0 / R)^3, pair list unchanged).  Cheap to make,
    since nothing is drawn but the size and the displacement."""
    sites = np.asarray(base.sites, dtype=np.int64)
    N = base.n_mono
    max_mono = N if max_mono is None else min(max_mono, N)
    rng = _rng(workload, r, KIND_STREAM)
    n = int(round(math.exp(rng.uniform(math.log(min_mono), math.log(max_mono)))))
    n = max(1, min(n, N))
    d2 = ((sites - sites.mean(axis=0)) ** 2).sum(axis=1)
    order = np.lexsort((np.arange(N), d2))[:n]
    order.sort()
    new_of = -np.ones(N, dtype=np.int64)
    new_of[order] = np.arange(n)
    nxv = base.n_occ.astype(np.int64) * base.n_vir
    psz = nxv[base.pairs[:, 0]] * nxv[base.pairs[:, 1]] if base.n_pair else np.zeros(0, np.int64)
    poff = np.concatenate([[0], np.cumsum(psz)])
    keep = np.flatnonzero((new_of[base.pairs[:, 0]] >= 0) & (new_of[base.pairs[:, 1]] >= 0)) \
        if base.n_pair else np.zeros(0, np.int64)
    pairs = new_of[base.pairs[keep]].astype(np.int32).reshape(-1, 2)
    mono = int(rng.integers(0, n))
    axis = int(rng.integers(0, 3))
    sign = 1.0 if rng.random() < 0.5 else -1.0
    pos = sites[order].astype(np.float64) * SPACING_A
    moved = pos.copy()
    moved[mono, axis] += sign * step_angstrom
    blocks = []
    for p, (x, y) in zip(keep, pairs):
        blk = base.v[poff[p]:poff[p + 1]]
        if x == mono or y == mono:
            r0 = float(np.linalg.norm(pos[x] - pos[y]))
            r1 = float(np.linalg.norm(moved[x] - moved[y]))
            blk = blk * (r0 / r1) ** 3
        blocks.append(blk)
    v = np.concatenate(blocks) if blocks else np.zeros(0)
    eoff = np.concatenate([[0], np.cumsum(base.n_occ.astype(np.int64) + base.n_vir)])
    koff = np.concatenate([[0], np.cumsum(nxv * nxv)])
    eps = np.concatenate([base.eps[eoff[x]:eoff[x + 1]] for x in order])
    k = np.concatenate([base.k[koff[x]:koff[x + 1]] for x in order])
    meta = dict(base.meta)
    meta.update(name=f"served-{r}", displacement=(mono, axis, sign * step_angstrom), carved_from=base.n_mono)
    return Problem(base.n_occ[order].copy(), base.n_vir[order].copy(), eps, k, pairs, v, sites[order], meta)


def singles_source(prob: Problem, *, workload: int | None = None, cluster: int | None = None,
                   sigma: float = SIGMA_W) -> np.ndarray:
    """Seeded stand-in for the embedding one-electron term w^a_i of each monomer
    (Eq. 26; its nuclear-attraction and Coulomb parts need geometries and AO
    integrals that are not available): w_X[i, a] ~ N(0, sigma^2), concatenated
    over monomers, row-major (o_X, v_X).  Keyed by the workload, the cluster and
    the monomer's lattice site (its index when the problem has no sites)."""
    wl = int(prob.meta.get("workload", 0) if workload is None else workload)
    cl = int(prob.meta.get("cluster", 0) if cluster is None else cluster)
    parts = []
    for x in range(prob.n_mono):
        key = prob.sites[x] if prob.sites is not None else (x, 0, 0)
        rng = _rng(wl, cl, KIND_SINGLES, *key)
        parts.append(rng.normal(0.0, sigma, size=prob.n_ov(x)))
    return np.concatenate(parts) if parts else np.zeros(0)


# ---------------------------------------------------------------------------
# intramonomer integral classes of the full monomer equation (Eq. 58)
# ---------------------------------------------------------------------------
_GROUP8 = [(0, 1, 2, 3), (1, 0, 2, 3), (0, 1, 3, 2), (1, 0, 3, 2),
           (2, 3, 0, 1), (3, 2, 0, 1), (2, 3, 1, 0), (3, 2, 1, 0)]
_GROUP4 = [(0, 1, 2, 3), (1, 0, 2, 3), (0, 1, 3, 2), (1, 0, 3, 2)]


def _symmetrised(rng, shape, group, sigma):
    """Normal draws averaged over a permutation group of the Mulliken indices
    (pr|qs), rescaled so that an element with distinct indices has standard
    deviation sigma."""
    g = rng.standard_normal(size=shape)
    s = np.zeros(shape)
    for perm in group:
        s += g.transpose(perm)
    return s * (sigma / math.sqrt(len(group)))


@dataclasses.dataclass
class LccdIntegrals:
    """Per-monomer integral classes of the intramonomer terms of Eq. 58, flat and
    concatenated over monomers (the layout the C ABI takes):

    w: W_X[a][b][c][d] = <ab|cd>, row-major (v, v, v, v)
    q: Q_X[i][j][k][l] = <ij|kl>, row-major (o, o, o, o)
    j: J_X[i][j][a][b] = <ia|jb> = (ij|ab), row-major (o, o, v, v)
    """
    n_occ: np.ndarray
    n_vir: np.ndarray
    w: np.ndarray
    q: np.ndarray
    j: np.ndarray

    def __post_init__(self):
        o = np.asarray(self.n_occ, dtype=np.int64)
        v = np.asarray(self.n_vir, dtype=np.int64)
        self.w_off = np.concatenate([[0], np.cumsum(v ** 4)])
        self.q_off = np.concatenate([[0], np.cumsum(o ** 4)])
        self.j_off = np.concatenate([[0], np.cumsum(o * o * v * v)])

    def w_of(self, x: int) -> np.ndarray:
        v = int(self.n_vir[x])
        return self.w[self.w_off[x]:self.w_off[x + 1]].reshape(v, v, v, v)

    def q_of(self, x: int) -> np.ndarray:
        o = int(self.n_occ[x])
        return self.q[self.q_off[x]:self.q_off[x + 1]].reshape(o, o, o, o)

    def j_of(self, x: int) -> np.ndarray:
        o, v = int(self.n_occ[x]), int(self.n_vir[x])
        return self.j[self.j_off[x]:self.j_off[x + 1]].reshape(o, o, v, v)

    def nbytes(self) -> int:
        return int(self.w.nbytes + self.q.nbytes + self.j.nbytes)

    def subset(self, monomers) -> "LccdIntegrals":
        ms = list(monomers)
        cat = lambda arr, off: np.concatenate([arr[off[x]:off[x + 1]] for x in ms]) if ms else np.zeros(0)
        return LccdIntegrals(np.asarray(self.n_occ)[ms], np.asarray(self.n_vir)[ms],
                             cat(self.w, self.w_off), cat(self.q, self.q_off), cat(self.j, self.j_off))


def concat_lccd(parts) -> LccdIntegrals:
    return LccdIntegrals(np.concatenate([p.n_occ for p in parts]), np.concatenate([p.n_vir for p in parts]),
                         np.concatenate([p.w for p in parts]), np.concatenate([p.q for p in parts]),
                         np.concatenate([p.j for p in parts]))


def lccd_integrals(prob: Problem, *, workload: int | None = None, cluster: int | None = None,
                   sigma: float = SIGMA_LCCD) -> LccdIntegrals:
    """Seeded stand-ins for the intramonomer integral classes (vv|vv), (oo|oo)
    and (oo|vv) of each monomer, drawn N(0, sigma^2) and symmetrised as real
    orbitals require within each class ((pr|qs) = (rp|qs) = (pr|sq) = (qs|pr)
    for (vv|vv) and (oo|oo); (ij|ab) = (ji|ab) = (ij|ba) for (oo|vv)).  Keyed by
    the workload, the cluster and the monomer's lattice site (its index when the
    problem has no sites)."""
    wl = int(prob.meta.get("workload", 0) if workload is None else workload)
    cl = int(prob.meta.get("cluster", 0) if cluster is None else cluster)
    ws, qs, js = [], [], []
    for x in range(prob.n_mono):
        o, v = int(prob.n_occ[x]), int(prob.n_vir[x])
        key = prob.sites[x] if prob.sites is not None else (x, 0, 0)
        rng = _rng(wl, cl, KIND_LCCD, *key)
        g_vv = _symmetrised(rng, (v, v, v, v), _GROUP8, sigma)     # (ac|bd)
        g_oo = _symmetrised(rng, (o, o, o, o), _GROUP8, sigma)     # (ik|jl)
        g_ov = _symmetrised(rng, (o, o, v, v), _GROUP4, sigma)     # (ij|ab)
        ws.append(np.ascontiguousarray(g_vv.transpose(0, 2, 1, 3)).ravel())   # <ab|cd> = (ac|bd)
        qs.append(np.ascontiguousarray(g_oo.transpose(0, 2, 1, 3)).ravel())   # <ij|kl> = (ik|jl)
        js.append(g_ov.ravel())                                               # <ia|jb> = (ij|ab)
    cat = lambda parts: np.concatenate(parts) if parts else np.zeros(0)
    return LccdIntegrals(prob.n_occ.copy(), prob.n_vir.copy(), cat(ws), cat(qs), cat(js))


def make_lccd_workload(name: str, coupling_scale: float = DEFAULT_COUPLING_SCALE, **kw):
    """A named cube with the intramonomer integral classes of the full monomer
    equation: K drawn at LCCD_K_SCALE x its sigma and (vv|vv), (oo|oo), (oo|vv)
    at SIGMA_LCCD.  Returns (problem, integrals)."""
    p = make_workload(name, coupling_scale=coupling_scale, k_scale=LCCD_K_SCALE, **kw)
    return p, lccd_integrals(p)


# ---------------------------------------------------------------------------
# dimer integral classes of the dimer-internal terms (Eq. 59)
# ---------------------------------------------------------------------------
KIND_DIMER = 6
SIGMA_DIMER = 0.01


@dataclasses.dataclass
class DimerIntegrals:
    """Per-pair integral classes of the dimer-internal terms of Eq. 59, flat and
    concatenated over the stored pairs (X = the first monomer of the pair), the
    layout the C ABI takes:

    w:  W_XY[a][b][a1][b1]   = <a b|a1 b1> = (a a1|b b1), (vX, vY, vX, vY)
    q:  Q_XY[i1][j1][i][j]   = <i1 j1|i j> = (i1 i|j1 j), (oX, oY, oX, oY)
    cx: C_X[i1][i][b][b1]    = (i1 i|b b1), X occupied and Y virtual, (oX, oX, vY, vY)
    cy: C_Y[j1][j][a][a1]    = (j1 j|a a1), Y occupied and X virtual, (oY, oY, vX, vX)
    """
    shapes: np.ndarray    # (n_pair, 4): oX, vX, oY, vY
    w: np.ndarray
    q: np.ndarray
    cx: np.ndarray
    cy: np.ndarray

    def __post_init__(self):
        sh = np.asarray(self.shapes, dtype=np.int64).reshape(-1, 4)
        ox, vx, oy, vy = sh[:, 0], sh[:, 1], sh[:, 2], sh[:, 3]
        off = lambda n: np.concatenate([[0], np.cumsum(n)]).astype(np.int64)
        self.w_off = off(vx * vy * vx * vy)
        self.q_off = off(ox * oy * ox * oy)
        self.cx_off = off(ox * ox * vy * vy)
        self.cy_off = off(oy * oy * vx * vx)

    @property
    def n_pair(self) -> int:
        return int(np.asarray(self.shapes).reshape(-1, 4).shape[0])

    def _sh(self, p):
        return (int(t) for t in np.asarray(self.shapes).reshape(-1, 4)[p])

    def w_of(self, p: int) -> np.ndarray:
        ox, vx, oy, vy = self._sh(p)
        return self.w[self.w_off[p]:self.w_off[p + 1]].reshape(vx, vy, vx, vy)

    def q_of(self, p: int) -> np.ndarray:
        ox, vx, oy, vy = self._sh(p)
        return self.q[self.q_off[p]:self.q_off[p + 1]].reshape(ox, oy, ox, oy)

    def cx_of(self, p: int) -> np.ndarray:
        ox, vx, oy, vy = self._sh(p)
        return self.cx[self.cx_off[p]:self.cx_off[p + 1]].reshape(ox, ox, vy, vy)

    def cy_of(self, p: int) -> np.ndarray:
        ox, vx, oy, vy = self._sh(p)
        return self.cy[self.cy_off[p]:self.cy_off[p + 1]].reshape(oy, oy, vx, vx)

    def nbytes(self) -> int:
        return int(self.w.nbytes + self.q.nbytes + self.cx.nbytes + self.cy.nbytes)


def dimer_integrals(prob: Problem, *, workload: int | None = None, cluster: int | None = None,
                    sigma: float = SIGMA_DIMER, workers: int = 1) -> DimerIntegrals:
    """Seeded stand-ins for the dimer classes (vX vX|vY vY), (oX oX|oY oY),
    (oX oX|vY vY) and (oY oY|vX vX) of every stored pair, drawn N(0, s^2) with
    s = sigma (R_nn / R)^3 like the pair blocks and symmetrised as real orbitals
    require within each charge distribution ((pr|qs) = (rp|qs) = (pr|sq)).  Keyed
    by the workload, the cluster and the two lattice sites, so workers > 1 (pairs
    drawn on that many threads into preallocated arrays) gives the same values."""
    wl = int(prob.meta.get("workload", 0) if workload is None else workload)
    cl = int(prob.meta.get("cluster", 0) if cluster is None else cluster)
    sites = prob.sites if prob.sites is not None else np.stack([np.arange(prob.n_mono), np.zeros(prob.n_mono),
                                                                np.zeros(prob.n_mono)], axis=1).astype(np.int64)
    P = prob.n_pair
    shapes = np.zeros((P, 4), dtype=np.int64)
    for p, (x, y) in enumerate(prob.pairs):
        shapes[p] = (int(prob.n_occ[x]), int(prob.n_vir[x]), int(prob.n_occ[y]), int(prob.n_vir[y]))
    ox, vx, oy, vy = (shapes[:, k] for k in range(4))
    offs = [np.concatenate([[0], np.cumsum(sz)]) for sz in (vx * vy * vx * vy, ox * oy * ox * oy,
                                                          ox * ox * vy * vy, oy * oy * vx * vx)]
    out = [np.empty(int(o[-1])) for o in offs]

    def one(p):
        x, y = (int(t) for t in prob.pairs[p])
        a, b, c, d = (int(t) for t in shapes[p])
        r = float(np.linalg.norm((np.asarray(sites[x]) - np.asarray(sites[y])).astype(np.float64))) or 1.0
        s = sigma / r ** 3
        rng = _rng(wl, cl, KIND_DIMER, *sites[x], *sites[y])
        g_vv = _symmetrised(rng, (b, b, d, d), _GROUP4, s)      # (a a1|b b1)
        g_oo = _symmetrised(rng, (a, a, c, c), _GROUP4, s)      # (i1 i|j1 j)
        g_ov = _symmetrised(rng, (a, a, d, d), _GROUP4, s)      # (i1 i|b b1)
        g_vo = _symmetrised(rng, (c, c, b, b), _GROUP4, s)      # (j1 j|a a1)
        for k, blk in enumerate((g_vv.transpose(0, 2, 1, 3), g_oo.transpose(0, 2, 1, 3), g_ov, g_vo)):
            out[k][offs[k][p]:offs[k][p + 1]] = blk.ravel()     # <a b|a1 b1>, <i1 j1|i j>, as drawn, as drawn

    if workers > 1 and P > 1:
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(max_workers=workers) as ex:
            list(ex.map(one, range(P)))
    else:
        for p in range(P):
            one(p)
    return DimerIntegrals(shapes.reshape(-1, 4), *out)


# named workloads with the dimer classes: the crystals with nearest-neighbour pairs only (the
# (vv|vv) class alone is 4.25 MB per pair at o = 5, v = 27)
DIMER_WORKLOADS = {
    "hf-3x3x3-c1": dict(workload=7, dims=(3, 3, 3), cutoff=1.0),
    "hf-10x10x10-c1": dict(workload=3, dims=(10, 10, 10), cutoff=1.0),
    # nearest and face-diagonal neighbours (squared lattice distance <= 2): 7,560 pairs
    "hf-10x10x10-c1.5": dict(workload=3, dims=(10, 10, 10), cutoff=1.5),
}


def make_dimer_workload(name: str, coupling_scale: float = DEFAULT_COUPLING_SCALE, workers: int = 1):
    """A named crystal with K at LCCD_K_SCALE x its sigma, the intramonomer classes
    and the dimer classes.  Returns (problem, intramonomer integrals, dimer integrals)."""
    spec = DIMER_WORKLOADS[name]
    p = make_lattice_problem(cubic_sites(*spec["dims"]), spec["cutoff"], workload=spec["workload"],
                             coupling_scale=coupling_scale, k_scale=LCCD_K_SCALE)
    p.meta["name"] = name
    return p, lccd_integrals(p), dimer_integrals(p, workers=workers)


# ---------------------------------------------------------------------------
# finite-displacement modes (Sec. IV.A: symmetric stretches of the molecules of
# a unit cell, five-point grid)
# ---------------------------------------------------------------------------
# sign patterns of the four cell molecules for the four stretch modes, in the
# spirit of S(Ag), S(B3u), S(B2u), S(B1g) of the orthorhombic cell
STRETCH_PATTERNS = {"Ag": (1, 1, 1, 1), "B3u": (1, -1, 1, -1), "B2u": (1, 1, -1, -1), "B1g": (1, -1, -1, 1)}


def central_cell(prob: Problem) -> np.ndarray:
    """Indices of the 2 x 2 x 1 block of monomers nearest the centre of the
    problem's lattice (the 'unit cell' whose energy is differentiated)."""
    sites = np.asarray(prob.sites, dtype=np.int64)
    lo = np.floor((sites.max(axis=0) - 1) / 2.0).astype(np.int64)
    want = [tuple(lo + np.array(d)) for d in ((0, 0, 0), (0, 1, 0), (1, 0, 0), (1, 1, 0))]
    index = {tuple(s): k for k, s in enumerate(sites)}
    return np.array([index[w] for w in want], dtype=np.int32)


def displacement_scales(prob: Problem, shifts: dict, points=(-2, -1, 1, 2), step_angstrom: float = 0.01):
    """Coupling factors (R0 / R)^3 of every pair that a displacement changes.

    shifts: monomer index -> unit direction (3-vector); at grid point s the
    monomer moves by s * step along it.  Returns (pair indices, factors
    [len(points)][n]) for the pairs with at least one moved monomer (the pair
    list of the undisplaced lattice is kept)."""
    pos = np.asarray(prob.sites, dtype=np.float64) * SPACING_A
    moved = np.zeros(prob.n_mono, dtype=bool)
    u = np.zeros((prob.n_mono, 3))
    for x, d in shifts.items():
        moved[int(x)] = True
        u[int(x)] = np.asarray(d, dtype=np.float64)
    idx = np.flatnonzero(moved[prob.pairs[:, 0]] | moved[prob.pairs[:, 1]]) if prob.n_pair else np.zeros(0, int)
    x, y = prob.pairs[idx, 0], prob.pairs[idx, 1]
    r0 = np.linalg.norm(pos[x] - pos[y], axis=1)
    out = np.empty((len(points), len(idx)))
    for k, s in enumerate(points):
        d = (pos[x] + s * step_angstrom * u[x]) - (pos[y] + s * step_angstrom * u[y])
        out[k] = (r0 / np.linalg.norm(d, axis=1)) ** 3
    return idx.astype(np.int64), out


def stretch_modes(prob: Problem, cell=None, axis: int = 0, step_angstrom: float = 0.01):
    """The four stretch modes of the cell: each cell monomer moved along `axis`
    with the sign of its pattern.  Returns [(name, pairs, factors[4][n])] for
    the grid points -2h, -h, +h, +2h."""
    cell = central_cell(prob) if cell is None else np.asarray(cell)
    e = np.zeros(3)
    e[axis] = 1.0
    modes = []
    for name, signs in STRETCH_PATTERNS.items():
        shifts = {int(c): sgn * e for c, sgn in zip(cell, signs)}
        pairs, f = displacement_scales(prob, shifts, step_angstrom=step_angstrom)
        modes.append((name, pairs, f))
    return modes


def scaled_problem(prob: Problem, pairs, factors) -> Problem:
    """A copy of prob with the blocks of the listed pairs multiplied by factors."""
    v = prob.v.copy()
    for p, f in zip(pairs, factors):
        v[prob.v_off[p]:prob.v_off[p + 1]] *= f
    return Problem(prob.n_occ, prob.n_vir, prob.eps, prob.k, prob.pairs, v, prob.sites, dict(prob.meta))
