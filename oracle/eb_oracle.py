"""CPU FP64 oracle of the embedded-boundary (cut-cell) elliptic problem —
TEST INFRASTRUCTURE ONLY (tests, smoke check, benchmark CPU leg).

The paper treats solid boundaries (the electrode) with an embedded-boundary
finite-volume formalism on Cartesian cells (Sec. 2, the discretisation list:
cut cells with volume fractions, second-order cell-centred elliptic
operators; Sec. 2.2: curved boundaries degrade multigrid convergence).  This
oracle states the discrete problem plainly and solves it with a sparse
direct solver.  The geometry (volume fractions kappa, face apertures, the
closest surface point of each boundary cell) is an input
(synth.geometry).

Per cell P with kappa_P > 0, integrated over the gas part of the cell and
divided by h^3:

  kappa_P a u_P + h^-2 sum_faces beta_f alpha_f (u_P - u_N)
      + h^-2 sum_{Dirichlet box faces} 2 beta_P alpha_f (u_P - g_face)
      + (beta_P A_P / h) dudn_P(u)                     = kappa_P f_P

- alpha_f: the face aperture; beta_f the harmonic mean of the two cells'
  beta (the cell permittivity, 1 if none);
- the embedded face: its area vector is fixed by the divergence theorem on
  the cut cell, A_P n_P = -sum_f alpha_f n_f h^2 over the six faces (n_f the
  outward unit normals), so that constant gradients are integrated
  exactly; A_P = |A_P n_P| (in units of h^2 below), n_P points out of the
  gas, nu = -n_P into it;
- dudn_P: the derivative of u along nu at the surface point x_b (given),
  where u = g_P: second-order one-sided differences from two points on the
  ray, x_1 = x_b + h nu and x_2 = x_b + 2 h nu, each valued by trilinear
  interpolation of the cell-centred unknowns (the 8 cell centres around the
  point; near the box faces the 8-cell block is shifted inside and the
  formula extrapolates):  dudn = [4 (u(x_1) - g) - (u(x_2) - g)] / (2 h);
- a cell with A_P = 0 has no embedded face.
Covered cells (kappa_P = 0) hold u_P = g_P: the row h^-2 u_P = h^-2 g_P.

The operator is not symmetric (the embedded-face rows reach cells along the
ray).  It is exact for linear u (all terms are exact for linear functions
and the embedded area closes the divergence theorem), which the pins use.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional, Sequence, Union

import numpy as np


@dataclass
class EBProblem:
    base: "object"              # synth.Problem: grid, a, f, eps (beta), box faces
    geom: "object"              # synth.geometry.Geometry
    g: Union[float, np.ndarray] = 1.0   # potential of the embedded surface: scalar or per cell
    # optional per-cell values on Dirichlet box faces (face index -> 2D array), overriding bc values
    face_values: Optional[dict] = None
    name: str = ""


def _harm(a, b):
    return 2.0 * a * b / (a + b)


def _gcell(prob: EBProblem, idx: np.ndarray) -> np.ndarray:
    if np.isscalar(prob.g):
        return np.full(np.shape(idx), float(prob.g))
    return np.asarray(prob.g, dtype=np.float64).reshape(-1)[idx]


def embedded_faces(prob: EBProblem):
    """Per boundary cell: area A (units h^2), inward normal nu, and the two
    trilinear stencils (indices [nb][2][8], weights [nb][2][8])."""
    q, G = prob.base, prob.geom
    nx, ny, nz = q.nx, q.ny, q.nz
    k, r = np.divmod(G.bidx, nx * ny)
    j, i = np.divmod(r, nx)
    # A n = -sum alpha_f n_f over the six faces (outward normals -e and +e)
    an = np.stack([
        -(G.ax[k, j, i + 1] - G.ax[k, j, i]),
        -(G.ay[k, j + 1, i] - G.ay[k, j, i]),
        -(G.az[k + 1, j, i] - G.az[k, j, i]),
    ], axis=1)
    A = np.linalg.norm(an, axis=1)
    nu = np.zeros_like(an)
    ok = A > 1e-12
    nu[ok] = -an[ok] / A[ok, None]
    nb = G.bidx.size
    idx = np.zeros((nb, 2, 8), dtype=np.int64)
    w = np.zeros((nb, 2, 8))
    centre = np.stack([i + 0.5, j + 0.5, k + 0.5], axis=1)   # units of h
    xb = centre + G.boff
    dims = np.array([nx, ny, nz])
    for m, dist in enumerate((1.0, 2.0)):
        pt = xb + dist * nu                        # units of h
        c = pt - 0.5                               # cell-index coordinates
        lo = np.floor(c).astype(np.int64)
        lo = np.clip(lo, 0, dims - 2)              # shift the 8-cell block inside the box
        t = c - lo                                 # may leave [0, 1]: extrapolation
        for o in range(8):
            ox, oy, oz = o & 1, (o >> 1) & 1, o >> 2
            wx = t[:, 0] if ox else 1.0 - t[:, 0]
            wy = t[:, 1] if oy else 1.0 - t[:, 1]
            wz = t[:, 2] if oz else 1.0 - t[:, 2]
            idx[:, m, o] = ((lo[:, 2] + oz) * ny + (lo[:, 1] + oy)) * nx + (lo[:, 0] + ox)
            w[:, m, o] = wx * wy * wz
    return A, nu, idx, w


def assemble(prob: EBProblem):
    """Sparse A (CSR, rows per unit volume) and b of the cut-cell problem."""
    import scipy.sparse as sp
    q, G = prob.base, prob.geom
    nx, ny, nz, h = q.nx, q.ny, q.nz, q.h
    n = nx * ny * nz
    ih2 = 1.0 / (h * h)
    beta = np.ones((nz, ny, nx)) if q.eps is None else np.asarray(q.eps, dtype=np.float64)
    kappa = G.kappa
    cov = (kappa <= 0).reshape(-1)
    flat = np.arange(n).reshape(nz, ny, nx)
    rows, cols, vals = [], [], []
    diag = np.zeros(n)
    b = np.where(cov, 0.0, (kappa * q.f).reshape(-1))
    diag += np.where(cov, 0.0, (kappa * q.a).reshape(-1))
    # interior faces along each axis: coefficient beta_f alpha_f / h^2, rows of uncovered cells only
    for axis, ap in ((0, G.ax[:, :, 1:-1]), (1, G.ay[:, 1:-1, :]), (2, G.az[1:-1])):
        sl_lo = [slice(None)] * 3
        sl_hi = [slice(None)] * 3
        sl_lo[2 - axis] = slice(0, -1)
        sl_hi[2 - axis] = slice(1, None)
        P, N = flat[tuple(sl_lo)].reshape(-1), flat[tuple(sl_hi)].reshape(-1)
        c = (ap * _harm(beta[tuple(sl_lo)], beta[tuple(sl_hi)]) * ih2).reshape(-1)
        for a_, b_ in ((P, N), (N, P)):
            keep = ~cov[a_] & (c != 0)
            np.add.at(diag, a_[keep], c[keep])
            rows.append(a_[keep])
            cols.append(b_[keep])
            vals.append(-c[keep])
    # box faces
    types, values = q.bc_types(), q.bc_values()
    for d in range(6):
        if types[d] != "D":
            continue
        axis, hi = d // 2, d % 2
        sl = [slice(None)] * 3
        sl[2 - axis] = -1 if hi else 0
        aps = (G.ax, G.ay, G.az)[axis]
        fsl = [slice(None)] * 3
        fsl[2 - axis] = -1 if hi else 0
        ap = aps[tuple(fsl)]
        P = flat[tuple(sl)].reshape(-1)
        c = (2.0 * beta[tuple(sl)] * ap * ih2).reshape(-1)
        gv = values[d] if not (prob.face_values and d in prob.face_values) else np.asarray(prob.face_values[d])
        gv = np.broadcast_to(gv, ap.shape).reshape(-1)
        keep = ~cov[P]
        np.add.at(diag, P[keep], c[keep])
        np.add.at(b, P[keep], (c * gv)[keep])
    # embedded faces
    A, nu, idx, w = embedded_faces(prob)
    gb = _gcell(prob, G.bidx)
    coef = beta.reshape(-1)[G.bidx] * A * ih2          # beta A / h  times 1/h from dudn
    for m, s in ((0, 2.0), (1, -0.5)):                  # dudn h = 2 (u1 - g) - (u2 - g) / 2
        rr = np.repeat(G.bidx, 8)
        rows.append(rr)
        cols.append(idx[:, m, :].reshape(-1))
        vals.append((coef[:, None] * s * w[:, m, :]).reshape(-1))
    b[G.bidx] += coef * 1.5 * gb
    # covered cells
    covi = np.flatnonzero(cov)
    diag[covi] = ih2
    b[covi] = ih2 * _gcell(prob, covi)
    rows.append(np.arange(n))
    cols.append(np.arange(n))
    vals.append(diag)
    Am = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    Am.sum_duplicates()
    return Am, b


def rhs_only(prob: EBProblem) -> np.ndarray:
    """The right-hand side b without assembling the operator (the same
    terms as assemble's b, for grids too large to assemble)."""
    q, G = prob.base, prob.geom
    nx, ny, nz, h = q.nx, q.ny, q.nz, q.h
    ih2 = 1.0 / (h * h)
    beta = np.ones((nz, ny, nx)) if q.eps is None else np.asarray(q.eps, dtype=np.float64)
    cov = G.kappa <= 0
    b = np.where(cov, 0.0, G.kappa * q.f)
    types, values = q.bc_types(), q.bc_values()
    for d in range(6):
        if types[d] != "D":
            continue
        axis, hi = d // 2, d % 2
        sl = [slice(None)] * 3
        sl[2 - axis] = -1 if hi else 0
        ap = (G.ax, G.ay, G.az)[axis][tuple(sl)]
        gv = values[d] if not (prob.face_values and d in prob.face_values) else np.asarray(prob.face_values[d])
        c = 2.0 * beta[tuple(sl)] * ap * ih2
        b[tuple(sl)] += np.where(cov[tuple(sl)], 0.0, c * gv)
    bf = b.reshape(-1)
    A, _, _, _ = embedded_faces(prob)
    coef = beta.reshape(-1)[G.bidx] * A * ih2
    bf[G.bidx] += coef * 1.5 * _gcell(prob, G.bidx)
    covi = np.flatnonzero(cov.reshape(-1))
    bf[covi] = ih2 * _gcell(prob, covi)
    return b


def solve(prob: EBProblem) -> np.ndarray:
    import scipy.sparse.linalg as spla
    Am, b = assemble(prob)
    q = prob.base
    return spla.spsolve(Am.tocsc(), b).reshape(q.nz, q.ny, q.nx)


def apply(prob: EBProblem, u: np.ndarray) -> np.ndarray:
    """A u (the operator without boundary data)."""
    Am, _ = assemble(prob)
    q = prob.base
    return (Am @ np.asarray(u, dtype=np.float64).reshape(-1)).reshape(q.nz, q.ny, q.nx)


def rhs(prob: EBProblem) -> np.ndarray:
    _, b = assemble(prob)
    q = prob.base
    return b.reshape(q.nz, q.ny, q.nx)


def residual(prob: EBProblem, u: np.ndarray):
    """(||b - A u||, ||b||), plain 2-norms over all rows."""
    Am, b = assemble(prob)
    r = b - Am @ np.asarray(u, dtype=np.float64).reshape(-1)
    return float(np.linalg.norm(r)), float(np.linalg.norm(b))


def residual_at(prob: EBProblem, u: np.ndarray, cells) -> np.ndarray:
    """b - A u at the given flat cell indices, one row at a time (for grids
    too large to assemble)."""
    q, G = prob.base, prob.geom
    nx, ny, nz, h = q.nx, q.ny, q.nz, q.h
    ih2 = 1.0 / (h * h)
    uf = np.asarray(u, dtype=np.float64).reshape(-1)
    beta = None if q.eps is None else np.asarray(q.eps, dtype=np.float64).reshape(-1)
    bet = (lambda p: 1.0) if beta is None else (lambda p: beta[p])
    kap = G.kappa.reshape(-1)
    f = np.asarray(q.f, dtype=np.float64).reshape(-1)
    types, values = q.bc_types(), q.bc_values()
    A, nu, idx, w = embedded_faces(prob)
    pos = {int(p): m for m, p in enumerate(G.bidx)}
    out = np.empty(len(cells))
    for t, P in enumerate(cells):
        P = int(P)
        k, r = divmod(P, nx * ny)
        j, i = divmod(r, nx)
        if kap[P] <= 0:
            gP = float(prob.g) if np.isscalar(prob.g) else float(np.asarray(prob.g).reshape(-1)[P])
            out[t] = ih2 * gP - ih2 * uf[P]
            continue
        bP = bet(P)
        acc = kap[P] * q.a * uf[P]
        rhs_ = kap[P] * f[P]
        faces = ((G.ax[k, j, i], i > 0, P - 1, 0), (G.ax[k, j, i + 1], i < nx - 1, P + 1, 1),
                 (G.ay[k, j, i], j > 0, P - nx, 2), (G.ay[k, j + 1, i], j < ny - 1, P + nx, 3),
                 (G.az[k, j, i], k > 0, P - nx * ny, 4), (G.az[k + 1, j, i], k < nz - 1, P + nx * ny, 5))
        for al, inside, N, d in faces:
            if inside:
                c = al * _harm(bP, bet(N)) * ih2
                acc += c * (uf[P] - uf[N])
            elif types[d] == "D":
                c = 2.0 * bP * al * ih2
                acc += c * uf[P]
                rhs_ += c * values[d]
        if P in pos:
            m = pos[P]
            coef = bP * A[m] * ih2
            acc += coef * (2.0 * (w[m, 0] * uf[idx[m, 0]]).sum() - 0.5 * (w[m, 1] * uf[idx[m, 1]]).sum())
            gP = float(prob.g) if np.isscalar(prob.g) else float(np.asarray(prob.g).reshape(-1)[P])
            rhs_ += coef * 1.5 * gP
        out[t] = rhs_ - acc
    return out
