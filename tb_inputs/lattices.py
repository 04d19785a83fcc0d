"""Seeded synthetic tight-binding lattices, returned as CSR matrices.

These are the inputs of the propagation: both the CPU oracle and the GPU
library receive the same arrays from here.  The module builds Hamiltonians
only; it performs none of the propagation arithmetic (no Chebyshev terms,
no Bessel coefficients, no correlation functions).

Conventions (TBPLaS 2.0, "Basic modeling"):
  * a hopping (R, i, j, t) means <i, cell 0 | H | j, cell R> = t, and every
    listed hopping is added together with its conjugate partner
    H_ji(-R) = conj(H_ij(R));
  * the graphene primitive cell has two p_z orbitals at fractional positions
    (0, 0) and (1/3, 1/3) of lattice vectors with a 60 degree angle,
    a = 0.246 nm, and three hoppings t = -2.7 eV: (0,0) 0->1, (1,0) 1->0,
    (0,1) 1->0.
Orbital index in a La x Lb supercell with periodic wrap:
  index = (a * Lb + b) * n_orb + o      (a slowest, o fastest).

Disorder, vacancies and sampled sites use numpy's PCG64 generator seeded with
the given seed; they are input data, not random numbers the method draws.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

# (dR_a, dR_b, orb_i, orb_j, t): one hopping term of a primitive cell.
Hop = Tuple[int, int, int, int, complex]

GRAPHENE_T = -2.7          # eV, nearest-neighbour hopping of the paper's graphene cell
BILAYER_GAMMA1 = 0.39      # eV, interlayer B1-A2 hopping of Bernal bilayer graphene


@dataclass
class PrimCell:
    """A primitive cell: orbital count, on-site energies and hopping terms, and
    its geometry (lattice vectors in nm, orbital positions as fractions of
    them), which the current and density operators need."""
    name: str
    n_orb: int
    hops: List[Hop]
    onsite: Tuple[float, ...] = ()
    vectors: Tuple[Tuple[float, float], Tuple[float, float]] = ((1.0, 0.0), (0.0, 1.0))
    positions: Tuple[Tuple[float, float], ...] = ()


GRAPHENE_A = 0.246         # nm, graphene lattice constant
_HEX = ((GRAPHENE_A, 0.0), (GRAPHENE_A / 2.0, GRAPHENE_A * 3.0 ** 0.5 / 2.0))


@dataclass
class Lattice:
    """A Hamiltonian in CSR form plus the description it was built from."""
    name: str
    n: int
    row_ptr: np.ndarray          # int64 [n+1]
    col: np.ndarray              # int32 [nnz], sorted within each row
    val: np.ndarray              # complex128 [nnz]
    cell: Optional[PrimCell] = None
    dims: Tuple[int, int] = (0, 0)
    clean: bool = True           # no disorder, no vacancies: periodic Bloch picture holds
    onsite: Optional[np.ndarray] = None     # float64 [n] disorder added on the diagonal
    kept: Optional[np.ndarray] = None       # original orbital index of each kept orbital
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def to_dense(self) -> np.ndarray:
        """Dense matrix (small lattices only)."""
        if self.n > 20000:
            raise ValueError("to_dense is for small lattices")
        h = np.zeros((self.n, self.n), dtype=np.complex128)
        rows = np.repeat(np.arange(self.n), np.diff(self.row_ptr))
        np.add.at(h, (rows, self.col.astype(np.int64)), self.val)
        return h

    def as_complex64(self) -> np.ndarray:
        return self.val.astype(np.complex64)


# ----------------------------------------------------------------------------
# primitive cells
# ----------------------------------------------------------------------------

def graphene_cell(t: float = GRAPHENE_T) -> PrimCell:
    """The paper's graphene cell: two orbitals, three listed hoppings."""
    return PrimCell("graphene", 2, [(0, 0, 0, 1, t), (1, 0, 1, 0, t), (0, 1, 1, 0, t)], (0.0, 0.0),
                    _HEX, ((0.0, 0.0), (1.0 / 3.0, 1.0 / 3.0)))


def bilayer_cell(t: float = GRAPHENE_T, gamma1: float = BILAYER_GAMMA1) -> PrimCell:
    """Bernal (AB) bilayer: orbitals A1, B1 (layer 1) and A2, B2 (layer 2).

    Layer 2 is layer 1 shifted by (1/3, 1/3): A2 sits above B1, B2 at (2/3, 2/3).
    gamma1 couples B1 and A2 of the same cell.
    """
    hops: List[Hop] = []
    for base in (0, 2):
        a, b = base, base + 1
        hops += [(0, 0, a, b, t), (1, 0, b, a, t), (0, 1, b, a, t)]
    hops.append((0, 0, 1, 2, gamma1))
    third = 1.0 / 3.0
    return PrimCell("bilayer_ab", 4, hops, (0.0,) * 4, _HEX,
                    ((0.0, 0.0), (third, third), (third, third), (2 * third, 2 * third)))


def square_cell(t: float = -1.0, t2: float = 0.1) -> PrimCell:
    """Square lattice, one orbital, nearest (t) and next-nearest (t2) hopping."""
    hops: List[Hop] = [(1, 0, 0, 0, t), (0, 1, 0, 0, t)]
    if t2 != 0.0:
        hops += [(1, 1, 0, 0, t2), (1, -1, 0, 0, t2)]
    return PrimCell("square" if t2 == 0.0 else "square_nnn", 1, hops, (0.0,), ((1.0, 0.0), (0.0, 1.0)),
                    ((0.0, 0.0),))


def honeycomb3_cell(t1: float = -2.7, t2: float = -0.2, t3: float = -0.18) -> PrimCell:
    """Honeycomb with first, second and third neighbours (graphene geometry).

    2nd neighbours join equal sublattices at cell offsets (1,0), (0,1), (1,-1);
    3rd neighbours join A(a,b) to B(a-1,b-1), B(a+1,b-1), B(a-1,b+1).
    """
    hops: List[Hop] = [(0, 0, 0, 1, t1), (1, 0, 1, 0, t1), (0, 1, 1, 0, t1)]
    for o in (0, 1):
        hops += [(1, 0, o, o, t2), (0, 1, o, o, t2), (1, -1, o, o, t2)]
    hops += [(-1, -1, 0, 1, t3), (1, -1, 0, 1, t3), (-1, 1, 0, 1, t3)]
    return PrimCell("honeycomb3", 2, hops, (0.0, 0.0), _HEX, ((0.0, 0.0), (1.0 / 3.0, 1.0 / 3.0)))


def cell_by_name(name: str) -> PrimCell:
    return {"graphene": graphene_cell, "bilayer_ab": bilayer_cell, "square_nnn": square_cell,
            "square": lambda: square_cell(t2=0.0), "honeycomb3": honeycomb3_cell}[name]()


# ----------------------------------------------------------------------------
# supercell construction
# ----------------------------------------------------------------------------

def _stencil(cell: PrimCell):
    """Per source orbital o: list of (dA, dB, o', value) including conjugates."""
    per_orb: List[List[Tuple[int, int, int, complex]]] = [[] for _ in range(cell.n_orb)]
    for (da, db, i, j, t) in cell.hops:
        per_orb[i].append((da, db, j, complex(t)))
        per_orb[j].append((-da, -db, i, complex(t).conjugate()))
    return per_orb


def supercell(cell: PrimCell, la: int, lb: int, *, disorder_w: float = 0.0, seed: int = 0,
              vacancy_p: float = 0.0, vacancy_seed: Optional[int] = None,
              name: Optional[str] = None, chunk_cells: int = 1 << 20) -> Lattice:
    """Periodic la x lb supercell of `cell` as CSR.

    disorder_w > 0 adds an on-site energy uniform in [-W/2, W/2] to every
    orbital (Anderson disorder; stored on the diagonal even where it is 0).
    vacancy_p > 0 deletes each orbital independently with that probability;
    kept orbitals are renumbered in their original order and hoppings to
    deleted orbitals are dropped.  Rows are built `chunk_cells` cells at a
    time, so the peak memory is the output plus one chunk.
    """
    if la < 1 or lb < 1:
        raise ValueError("supercell dims must be >= 1")
    n_orb = cell.n_orb
    n = la * lb * n_orb
    per_orb = _stencil(cell)
    onsite_cell = np.asarray(cell.onsite if cell.onsite else (0.0,) * n_orb, dtype=np.float64)
    has_diag = disorder_w > 0.0 or np.any(onsite_cell != 0.0)
    # rows of different orbitals may hold different counts: pad to the max, drop padding later
    kmax = max(len(s) + (1 if has_diag else 0) for s in per_orb)

    onsite = None
    if disorder_w > 0.0:
        rng = np.random.default_rng(seed)
        onsite = rng.uniform(-0.5 * disorder_w, 0.5 * disorder_w, size=n)
    kept = None
    newidx = None
    if vacancy_p > 0.0:
        vrng = np.random.default_rng(seed if vacancy_seed is None else vacancy_seed)
        keep_mask = vrng.random(n) >= vacancy_p
        kept = np.nonzero(keep_mask)[0]
        newidx = np.full(n, -1, dtype=np.int64)
        newidx[kept] = np.arange(kept.size, dtype=np.int64)
        del keep_mask

    if kmax > 16:
        raise ValueError("at most 16 entries per row")
    vtab = np.zeros((n_orb, 16), dtype=np.complex128)     # value of (orbital, slot)
    ptab = np.zeros((n_orb, 16), dtype=bool)              # slot holds an entry
    dslot = np.full(n_orb, -1, dtype=np.int64)            # slot of the diagonal
    for o in range(n_orb):
        for k, (_, _, _, v) in enumerate(per_orb[o]):
            vtab[o, k] = v
            ptab[o, k] = True
        if has_diag:
            k = len(per_orb[o])
            vtab[o, k] = onsite_cell[o]
            ptab[o, k] = True
            dslot[o] = k

    counts_parts, col_parts, val_parts = [], [], []
    ncell = la * lb
    for c0 in range(0, ncell, chunk_cells):
        c1 = min(ncell, c0 + chunk_cells)
        cells = np.arange(c0, c1, dtype=np.int64)
        ca, cb = cells // lb, cells % lb
        m = c1 - c0
        rows = np.arange(c0 * n_orb, c1 * n_orb, dtype=np.int64)
        # sort each row by column through packed keys (column << 4 | slot), then
        # read the values back from the per-(orbital, slot) table
        keys = np.empty((m, n_orb, kmax), dtype=np.int64)
        for o in range(n_orb):
            for k in range(kmax):
                if k < len(per_orb[o]):
                    da, db, o2, _ = per_orb[o][k]
                    cc = (((ca + da) % la) * lb + ((cb + db) % lb)) * n_orb + o2
                else:                               # diagonal slot, or padding pointing at self
                    cc = cells * n_orb + o
                keys[:, o, k] = (cc << 4) | k
        keys = np.sort(keys.reshape(-1, kmax), axis=1)
        slot = keys & 15
        cols = keys >> 4
        del keys
        orb = (rows % n_orb)[:, None]
        vals = vtab[orb, slot]
        if onsite is not None:
            dg = slot == dslot[orb]
            vals = vals + np.where(dg, onsite[rows][:, None], 0.0)
        pres = ptab[orb, slot]
        del slot, orb
        if kmax > 1 and np.any((cols[:, 1:] == cols[:, :-1]) & pres[:, 1:] & pres[:, :-1]):
            if ncell > chunk_cells:
                raise ValueError("duplicate hoppings need a small supercell")
            return _supercell_slow(cols, vals, pres, n, cell, la, lb, onsite,
                                   None if newidx is None else newidx >= 0, kept, name, disorder_w)
        if newidx is not None:
            rk = newidx[rows] >= 0
            cols, vals, pres = cols[rk], vals[rk], pres[rk]
            pres &= newidx[cols] >= 0
            cols = newidx[cols]
            cols[~pres] = 0
        counts_parts.append(pres.sum(axis=1))
        col_parts.append(cols[pres].astype(np.int32))
        val_parts.append(vals[pres])
        del cols, vals, pres
    counts = np.concatenate(counts_parts)
    n_new = counts.size
    row_ptr = np.zeros(n_new + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    col = np.concatenate(col_parts) if len(col_parts) > 1 else col_parts[0]
    del col_parts
    val = np.concatenate(val_parts) if len(val_parts) > 1 else val_parts[0]
    del val_parts
    return Lattice(name or f"{cell.name}_{la}x{lb}", n_new, row_ptr, col, val, cell, (la, lb),
                   clean=(disorder_w == 0.0 and vacancy_p == 0.0), onsite=onsite, kept=kept,
                   meta={"disorder_w": disorder_w, "seed": seed, "vacancy_p": vacancy_p})


def _supercell_slow(cols, vals, pres, n, cell, la, lb, onsite, keep_mask, kept, name, disorder_w):
    """Duplicate-column path for very small supercells: sum coincident entries."""
    import scipy.sparse as sp
    rows = np.repeat(np.arange(n), cols.shape[1]).reshape(cols.shape)
    r, c, v = rows[pres], cols[pres], vals[pres]
    m = sp.coo_matrix((v, (r, c)), shape=(n, n)).tocsr()
    m.sum_duplicates()
    if kept is not None:
        m = m[kept][:, kept].tocsr()
        m.sum_duplicates()
    m.sort_indices()
    return Lattice(name or f"{cell.name}_{la}x{lb}", m.shape[0], m.indptr.astype(np.int64),
                   m.indices.astype(np.int32), m.data.astype(np.complex128), cell, (la, lb),
                   clean=(disorder_w == 0.0 and keep_mask is None), onsite=onsite, kept=kept,
                   meta={"disorder_w": disorder_w})


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------

def graphene(la: int, lb: Optional[int] = None, *, disorder_w: float = 0.0, seed: int = 0) -> Lattice:
    lb = la if lb is None else lb
    return supercell(graphene_cell(), la, lb, disorder_w=disorder_w, seed=seed)


def bilayer(la: int, lb: Optional[int] = None, *, disorder_w: float = 0.0, seed: int = 0) -> Lattice:
    lb = la if lb is None else lb
    return supercell(bilayer_cell(), la, lb, disorder_w=disorder_w, seed=seed)


def square(la: int, lb: Optional[int] = None, *, t: float = -1.0, t2: float = 0.1,
           disorder_w: float = 0.0, seed: int = 0) -> Lattice:
    lb = la if lb is None else lb
    return supercell(square_cell(t, t2), la, lb, disorder_w=disorder_w, seed=seed)


def honeycomb3(la: int, lb: Optional[int] = None, *, vacancy_p: float = 0.0, seed: int = 0) -> Lattice:
    lb = la if lb is None else lb
    return supercell(honeycomb3_cell(), la, lb, vacancy_p=vacancy_p, seed=seed)


def sample_sites(n: int, count: int, seed: int) -> np.ndarray:
    """`count` distinct orbital indices in [0, n), sorted (LDOS sampling sites)."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n, size=min(count, n), replace=False)).astype(np.int64)


def rescale_for(lat: Lattice) -> float:
    """Default energy rescale for the named workloads (eV)."""
    base = lat.cell.name if lat.cell is not None else lat.name
    return {"graphene": 9.0, "bilayer_ab": 9.0, "square_nnn": 4.5, "square": 4.5,
            "honeycomb3": 10.0}.get(base, 9.0)


def state_from_sites(n: int, sites: Sequence[int]) -> np.ndarray:
    """A normalized state with equal real amplitude on the given sites."""
    psi = np.zeros(n, dtype=np.complex128)
    s = np.asarray(sites, dtype=np.int64)
    psi[s] = 1.0 / np.sqrt(s.size)
    return psi


# ----------------------------------------------------------------------------
# operators built from the geometry (inputs of the response functions)
# ----------------------------------------------------------------------------

def _cell_coords(lat: Lattice, idx: np.ndarray):
    """(cell a, cell b, orbital) of stored orbitals `idx` (original numbering)."""
    cell = lat.cell
    orig = idx if lat.kept is None else lat.kept[idx]
    la, lb = lat.dims
    c, o = np.divmod(orig, cell.n_orb)
    ca, cb = np.divmod(c, lb)
    return ca, cb, o


def positions(lat: Lattice) -> np.ndarray:
    """Cartesian position (nm) of every orbital, float64 [n, 2], cells unwrapped."""
    cell = lat.cell
    ca, cb, o = _cell_coords(lat, np.arange(lat.n, dtype=np.int64))
    v = np.asarray(cell.vectors, dtype=np.float64)
    f = np.asarray(cell.positions, dtype=np.float64)
    frac = np.stack([ca + f[o, 0], cb + f[o, 1]], axis=1)
    return frac @ v


def hop_displacements(lat: Lattice) -> np.ndarray:
    """Displacement r_j + R - r_i (nm) of every stored entry H_ij, float64 [nnz, 2],
    with the periodic image chosen by the shortest cell offset (needs la, lb >= 3)."""
    cell = lat.cell
    la, lb = lat.dims
    if la < 3 or lb < 3:
        raise ValueError("hop displacements need at least 3 x 3 cells")
    rows = np.repeat(np.arange(lat.n, dtype=np.int64), np.diff(lat.row_ptr))
    ra, rb, ro = _cell_coords(lat, rows)
    ca, cb, co = _cell_coords(lat, lat.col.astype(np.int64))
    da = (ca - ra + la // 2) % la - la // 2
    db = (cb - rb + lb // 2) % lb - lb // 2
    f = np.asarray(cell.positions, dtype=np.float64)
    frac = np.stack([da + f[co, 0] - f[ro, 0], db + f[co, 1] - f[ro, 1]], axis=1)
    return frac @ np.asarray(cell.vectors, dtype=np.float64)


def current_operator(lat: Lattice, direction=(1.0, 0.0)) -> Lattice:
    """J = i [H, x.u] for the unit direction u: entries i (d_ij . u) H_ij on the
    sparsity of H (hbar = e = 1; eV nm).  Hermitian when H is."""
    u = np.asarray(direction, dtype=np.float64)
    d = hop_displacements(lat) @ u
    return Lattice(f"current_{lat.name}", lat.n, lat.row_ptr.copy(), lat.col.copy(), 1j * d * lat.val,
                   cell=lat.cell, dims=lat.dims, clean=lat.clean, kept=lat.kept,
                   meta={"operator": "current", "direction": tuple(u)})


def density_operator(lat: Lattice, q=(0.0, 0.0)) -> Lattice:
    """rho_q = sum_i exp(i q . r_i) |i><i| (q in 1/nm), as a diagonal CSR."""
    r = positions(lat)
    vals = np.exp(1j * (r @ np.asarray(q, dtype=np.float64)))
    return Lattice(f"density_{lat.name}", lat.n, np.arange(lat.n + 1, dtype=np.int64),
                   np.arange(lat.n, dtype=np.int32), vals.astype(np.complex128), cell=lat.cell, dims=lat.dims,
                   clean=lat.clean, kept=lat.kept, meta={"operator": "density", "q": tuple(q)})


def area_per_orbital(lat: Lattice) -> float:
    """Sample area (nm^2) divided by the number of orbitals."""
    v = np.asarray(lat.cell.vectors, dtype=np.float64)
    la, lb = lat.dims
    return abs(np.linalg.det(v)) * la * lb / lat.n
