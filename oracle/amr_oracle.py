"""CPU FP64 oracle of the composite (two-level AMR) elliptic problem — TEST
INFRASTRUCTURE ONLY (tests, smoke check, benchmark CPU leg).

The paper solves its elliptic equations on an adaptive hierarchy of Cartesian
patches (Secs. 2-4: a base grid refined by patches of 16^3-32^3 cells, ratio
2 or 4) with the second-order cell-centred discretisation of item (ii)-(iii).
This oracle states the composite discrete problem of a base grid plus
refinement-ratio-2 patches and solves it by plain means: it assembles the
sparse matrix cell by cell and calls a sparse direct solver.

Composite grid: the base grid (nx*ny*nz cells of side h, the box faces'
conditions of the single-grid problem) and boxes of the level-1 index space
(2nx*2ny*2nz cells of side h/2), given as fine cell ranges [lo, hi) per axis
with even bounds.  Boxes stay at least one coarse cell away from the box
faces and from each other.  Unknowns: the base cells no box covers, and every
fine cell.

Equations (per unit volume, a u - div(beta grad u) = f):
- between two cells of one level: the single-grid stencil (harmonic-mean face
  coefficient, spacing of that level);
- a fine cell F beside the coarse-fine interface sees a ghost value G beyond
  its face: G = F/3 + 2/3 C~, where C~ is the coarse value of the cell C that
  holds the ghost, moved to the ghost's tangential position by central
  differences of C's tangential neighbours, C~ = C + sum_t s_t (C_{+t} -
  C_{-t}) / 8 (s_t = -1 or +1 for the ghost in the lower or upper half of C
  along t).  G lies on the line from F's centre (h_f/2 inside) to C~'s point
  (h_f outside, C's centre plane), so G is exact for linear functions.  The
  face term is beta_i (F - G) / h_f^2 with beta_i the harmonic mean of the two
  cells' coefficients;
- a coarse cell C beside a patch takes, for that face, the sum of the four
  fine fluxes through it (refluxing): beta_i (G_i - F_i) / h_f * h_f^2 / h_c^3
  per sub-face, so the composite operator is conservative;
- Dirichlet and Neumann box faces as on a single grid (base level only).

The system is not symmetric (the ghost values couple coarse neighbours); its
solution is unique (an M-matrix-like diffusion operator with a > 0 or a
Dirichlet face)."""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

Box = Tuple[Tuple[int, int, int], Tuple[int, int, int]]  # (lo, hi), x y z, fine indices


@dataclass
class Composite:
    base: "object"                       # synth.Problem: the base grid and its box faces
    boxes: List[Box]
    f_fine: List[np.ndarray]             # per box [nz][ny][nx] of the fine cells
    eps_fine: Optional[List[np.ndarray]] = None  # per box, or None (beta = 1 on the patches)
    name: str = ""

    def shape(self, p: int) -> Tuple[int, int, int]:
        lo, hi = self.boxes[p]
        return (hi[2] - lo[2], hi[1] - lo[1], hi[0] - lo[0])


def check_boxes(nx: int, ny: int, nz: int, boxes: Sequence[Box]) -> None:
    """Raise ValueError unless every box has even bounds, lies at least one
    coarse cell inside the domain, and keeps one coarse cell from the others."""
    dims = (nx, ny, nz)
    for lo, hi in boxes:
        for d in range(3):
            if lo[d] % 2 or hi[d] % 2 or hi[d] <= lo[d]:
                raise ValueError(f"box {lo}-{hi}: bounds must be even and hi > lo")
            if lo[d] < 2 or hi[d] > 2 * dims[d] - 2:
                raise ValueError(f"box {lo}-{hi}: must stay one coarse cell inside the domain")
    for a in range(len(boxes)):
        for b in range(a + 1, len(boxes)):
            (l1, h1), (l2, h2) = boxes[a], boxes[b]
            if all(l1[d] - 2 < h2[d] and l2[d] < h1[d] + 2 for d in range(3)):
                raise ValueError(f"boxes {a} and {b} are less than one coarse cell apart")


def coverage(nx: int, ny: int, nz: int, boxes: Sequence[Box]) -> np.ndarray:
    """[nz][ny][nx] int array: the box covering each base cell, or -1."""
    m = -np.ones((nz, ny, nx), dtype=np.int64)
    for p, (lo, hi) in enumerate(boxes):
        m[lo[2] // 2:hi[2] // 2, lo[1] // 2:hi[1] // 2, lo[0] // 2:hi[0] // 2] = p
    return m


def _harm(a, b):
    return 2.0 * a * b / (a + b)


class _Index:
    """Unknown numbering: uncovered base cells first, then each box's cells
    in C order."""

    def __init__(self, comp: Composite):
        q = comp.base
        self.comp = comp
        self.mask = coverage(q.nx, q.ny, q.nz, comp.boxes)
        self.base_id = -np.ones(self.mask.shape, dtype=np.int64)
        unc = self.mask < 0
        self.base_id[unc] = np.arange(int(unc.sum()))
        self.n = int(unc.sum())
        self.off = []
        for p in range(len(comp.boxes)):
            self.off.append(self.n)
            self.n += int(np.prod(comp.shape(p)))

    def fine(self, p: int, i: int, j: int, k: int) -> int:
        """Unknown of fine cell (i, j, k) (global fine indices) of box p."""
        lo, hi = self.comp.boxes[p]
        nzp, nyp, nxp = self.comp.shape(p)
        return self.off[p] + ((k - lo[2]) * nyp + (j - lo[1])) * nxp + (i - lo[0])


class _Rows:
    """The equations of the composite problem, one row at a time: the
    unknowns and weights of a row and its right-hand side."""

    steps = [(-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]

    def __init__(self, comp: Composite):
        q = comp.base
        check_boxes(q.nx, q.ny, q.nz, comp.boxes)
        self.comp, self.q = comp, q
        self.ix = _Index(comp)
        self.hc, self.hf = q.h, 0.5 * q.h
        self.beta_c = np.ones(q.shape) if q.eps is None else np.asarray(q.eps, dtype=np.float64)
        self.beta_f = [np.ones(comp.shape(p)) if comp.eps_fine is None
                       else np.asarray(comp.eps_fine[p], dtype=np.float64) for p in range(len(comp.boxes))]
        self.types, self.vals = q.bc_types(), q.bc_values()

    def ghost_terms(self, p, fi, fj, fk, d, coef):
        """coef * G expressed through unknowns, for the ghost beyond face d of
        fine cell (fi, fj, fk) of box p: a list of (unknown, weight)."""
        ix = self.ix
        di, dj, dk = self.steps[d]
        gi, gj, gk = fi + di, fj + dj, fk + dk               # ghost (fine indices)
        C = (gi // 2, gj // 2, gk // 2)                      # coarse cell holding it
        axis = d // 2
        terms = [(ix.fine(p, fi, fj, fk), coef / 3.0)]       # F / 3
        ct = 2.0 / 3.0 * coef
        terms.append((ix.base_id[C[2], C[1], C[0]], ct))    # 2/3 C
        g = (gi, gj, gk)
        for t in range(3):
            if t == axis:
                continue
            s = 1.0 if g[t] % 2 else -1.0
            up, dn = list(C), list(C)
            up[t] += 1
            dn[t] -= 1
            for cc, w in ((up, 1.0), (dn, -1.0)):
                uid = ix.base_id[cc[2], cc[1], cc[0]]
                assert uid >= 0, "tangential neighbour of a ghost is covered"
                terms.append((uid, ct * s * w / 8.0))
        return terms

    def base_row(self, I, J, K):
        """(terms, rhs) of uncovered base cell (I, J, K)."""
        q, ix, comp = self.q, self.ix, self.comp
        ic2, hf = 1.0 / self.hc**2, self.hf
        r = ix.base_id[K, J, I]
        bC = self.beta_c[K, J, I]
        terms = [(r, q.a)]
        rhs = q.f[K, J, I]
        for d, (di, dj, dk) in enumerate(self.steps):
            N = (I + di, J + dj, K + dk)
            if not (0 <= N[0] < q.nx and 0 <= N[1] < q.ny and 0 <= N[2] < q.nz):
                if self.types[d] == "D":
                    terms.append((r, 2.0 * bC * ic2))
                    rhs += 2.0 * bC * ic2 * self.vals[d]
                continue
            pn = ix.mask[N[2], N[1], N[0]]
            if pn < 0:
                bf = _harm(bC, self.beta_c[N[2], N[1], N[0]])
                terms += [(r, bf * ic2), (ix.base_id[N[2], N[1], N[0]], -bf * ic2)]
                continue
            # coarse-fine face: the four fine fluxes (refluxing)
            axis = d // 2
            fn = [2 * N[0], 2 * N[1], 2 * N[2]]
            if di + dj + dk < 0:  # the fine layer of N beside C is its last one
                fn[axis] += 1
            tang = [t for t in range(3) if t != axis]
            for o1 in range(2):
                for o2 in range(2):
                    f = list(fn)
                    f[tang[0]] += o1
                    f[tang[1]] += o2
                    lo = comp.boxes[pn][0]
                    bF = self.beta_f[pn][f[2] - lo[2], f[1] - lo[1], f[0] - lo[0]]
                    w = _harm(bF, bC) / (8.0 * hf * hf)  # beta_i / h_f * h_f^2 / h_c^3
                    # + w (G - F), with G the ghost of F beyond the face towards C
                    terms += self.ghost_terms(pn, f[0], f[1], f[2], d ^ 1, w)
                    terms.append((ix.fine(pn, *f), -w))
        return terms, rhs

    def fine_row(self, p, i, j, k):
        """(terms, rhs) of fine cell (i, j, k) (global fine indices) of box p."""
        ix, comp = self.ix, self.comp
        if2 = 1.0 / self.hf**2
        lo, hi = comp.boxes[p]
        r = ix.fine(p, i, j, k)
        bF = self.beta_f[p][k - lo[2], j - lo[1], i - lo[0]]
        terms = [(r, self.q.a)]
        rhs = comp.f_fine[p][k - lo[2], j - lo[1], i - lo[0]]
        for d, (di, dj, dk) in enumerate(self.steps):
            n = (i + di, j + dj, k + dk)
            if all(lo[e] <= n[e] < hi[e] for e in range(3)):
                bf = _harm(bF, self.beta_f[p][n[2] - lo[2], n[1] - lo[1], n[0] - lo[0]])
                terms += [(r, bf * if2), (ix.fine(p, *n), -bf * if2)]
                continue
            C = (n[0] // 2, n[1] // 2, n[2] // 2)
            bi = _harm(bF, self.beta_c[C[2], C[1], C[0]])
            # beta_i (F - G) / h_f^2
            terms.append((r, bi * if2))
            terms += self.ghost_terms(p, i, j, k, d, -bi * if2)
        return terms, rhs


def assemble(comp: Composite):
    """Sparse A (CSR, per-volume rows) and b of the composite problem."""
    import scipy.sparse as sp
    R = _Rows(comp)
    q, ix = comp.base, R.ix
    rows, cols, data = [], [], []
    b = np.zeros(ix.n)

    def put(r, terms, rhs):
        for c, v in terms:
            rows.append(r)
            cols.append(c)
            data.append(v)
        b[r] += rhs

    for K in range(q.nz):
        for J in range(q.ny):
            for I in range(q.nx):
                r = ix.base_id[K, J, I]
                if r >= 0:
                    put(r, *R.base_row(I, J, K))
    for p, (lo, hi) in enumerate(comp.boxes):
        for k in range(lo[2], hi[2]):
            for j in range(lo[1], hi[1]):
                for i in range(lo[0], hi[0]):
                    put(ix.fine(p, i, j, k), *R.fine_row(p, i, j, k))
    A = sp.csr_matrix((data, (rows, cols)), shape=(ix.n, ix.n))
    A.sum_duplicates()
    return A, b, ix


def residual_at(comp: Composite, base: np.ndarray, fine: Sequence[np.ndarray], cells) -> np.ndarray:
    """b - A u at sampled cells, one row at a time (for grids too large to
    assemble): cells are ("c", I, J, K) for uncovered base cells or
    ("f", p, i, j, k) for fine cells (global fine indices)."""
    R = _Rows(comp)
    u = pack(comp, base, fine, R.ix)
    out = np.empty(len(cells))
    for n, c in enumerate(cells):
        terms, rhs = R.base_row(*c[1:]) if c[0] == "c" else R.fine_row(*c[1:])
        out[n] = rhs - sum(w * u[col] for col, w in terms)
    return out


def unpack(comp: Composite, u: np.ndarray, ix: "_Index"):
    """(base array with covered cells set to the mean of their 8 children,
    list of fine arrays) from the unknown vector."""
    q = comp.base
    base = np.zeros(q.shape)
    unc = ix.mask < 0
    base[unc] = u[ix.base_id[unc]]
    fine = []
    for p in range(len(comp.boxes)):
        nzp, nyp, nxp = comp.shape(p)
        a = u[ix.off[p]:ix.off[p] + nzp * nyp * nxp].reshape(nzp, nyp, nxp)
        fine.append(a.copy())
        lo, hi = comp.boxes[p]
        avg = a.reshape(nzp // 2, 2, nyp // 2, 2, nxp // 2, 2).mean(axis=(1, 3, 5))
        base[lo[2] // 2:hi[2] // 2, lo[1] // 2:hi[1] // 2, lo[0] // 2:hi[0] // 2] = avg
    return base, fine


def pack(comp: Composite, base: np.ndarray, fine: Sequence[np.ndarray], ix: "_Index") -> np.ndarray:
    u = np.zeros(ix.n)
    unc = ix.mask < 0
    u[ix.base_id[unc]] = base[unc]
    for p in range(len(comp.boxes)):
        u[ix.off[p]:ix.off[p] + fine[p].size] = np.asarray(fine[p]).reshape(-1)
    return u


def solve(comp: Composite):
    """The composite solution by a sparse direct solve: (base, [fine])."""
    import scipy.sparse.linalg as spla
    A, b, ix = assemble(comp)
    u = spla.spsolve(A.tocsc(), b)
    return unpack(comp, u, ix)


def apply(comp: Composite, base: np.ndarray, fine: Sequence[np.ndarray], homogeneous: bool = True):
    """A u of the composite operator ((base, [fine]) per-volume, covered base
    cells 0), without the Dirichlet values (homogeneous=True) or as
    A u - b + f (with them: the residual's operator part)."""
    A, b, ix = assemble(comp)
    y = A @ pack(comp, base, fine, ix)
    out_b, out_f = unpack(comp, y, ix)
    out_b[ix.mask >= 0] = 0.0
    return out_b, out_f


def residual(comp: Composite, base: np.ndarray, fine: Sequence[np.ndarray]):
    """(||b - A u||, ||b||) in the volume-weighted L2 norm over the unknowns."""
    A, b, ix = assemble(comp)
    r = b - A @ pack(comp, base, fine, ix)
    w = np.where(np.arange(ix.n) < ix.off[0] if ix.off else np.ones(ix.n, bool), comp.base.h**3,
                 (0.5 * comp.base.h) ** 3)
    return float(np.sqrt(np.sum(w * r * r))), float(np.sqrt(np.sum(w * b * b)))
