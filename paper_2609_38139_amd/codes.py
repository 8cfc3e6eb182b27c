"""Parity-check matrices of the code families the decoder is run on.

This module builds inputs only: the X-check matrix ``H`` (whose Tanner graph
the decoder runs on) and the commuting stabiliser matrix ``G`` (``H_Z`` for
Z noise) used by the homology test of the decoding-success definition
(Preliminaries, conditions (1) and (2)). It holds none of the decoder's
arithmetic and is shared by the HIP path and the CPU oracle's tests.

Index conventions (fixed; both the library and the tests rely on them):

* Cyclic shift ``S_k[i, j] = 1`` iff ``j = i + 1 (mod k)``. Group-algebra
  codes on ``Z_l x Z_m`` index the pair ``(i, j)`` as ``i*m + j`` with
  ``x = S_l (x) I_m`` and ``y = I_l (x) S_m``; ``H_X = [A | B]`` and
  ``H_Z = [B^T | A^T]`` (bivariate-bicycle section).
* 2D toric code of size L: the group-algebra code with ``A = 1 + x``,
  ``B = 1 + y`` (footnote of the bivariate-bicycle section). Qubits
  ``0..L^2-1`` form the A block, ``L^2..2L^2-1`` the B block; check ``i*L+j``
  is a vertex of weight 4; every qubit has degree 2.
* 3D toric code of size L: vertex ``(x, y, z)`` has index ``x + L*(y + L*z)``;
  edge ``e_a(v)`` (a = 0, 1, 2) joins ``v`` to ``v + a_hat`` and has index
  ``a*L^3 + v``; face ``f_t(v)`` for the pair ``(a, b)`` = (0,1), (0,2), (1,2)
  (t = 0, 1, 2) has index ``t*L^3 + v`` and edges
  ``{e_a(v), e_b(v), e_a(v + b_hat), e_b(v + a_hat)}``. The point-like sector
  checks vertices (weight 6); the membrane-like sector checks faces (weight 4,
  qubit degree 4).
* Repetition code of d bits: check j joins bits j and j+1 (mod d when
  periodic); it has no commuting stabilisers (G is empty).

Matrices are returned in CSR form (``rowptr``, ``col``; int32; columns strictly
ascending within a row), which is the form the C ABI takes.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class CSR:
    """A 0/1 matrix in compressed-sparse-row form."""

    rows: int
    cols: int
    rowptr: np.ndarray  # int32 [rows + 1]
    col: np.ndarray  # int32 [nnz]

    @staticmethod
    def from_rows(rows: int, cols: int, row_lists) -> "CSR":
        rowptr = np.zeros(rows + 1, dtype=np.int32)
        parts = []
        for r, lst in enumerate(row_lists):
            # an entry that appears twice cancels over GF(2)
            vals, counts = np.unique(np.asarray(lst, dtype=np.int64) % cols, return_counts=True)
            a = vals[counts % 2 == 1]
            parts.append(a.astype(np.int32))
            rowptr[r + 1] = rowptr[r] + len(a)
        col = np.concatenate(parts) if parts else np.zeros(0, dtype=np.int32)
        return CSR(rows, cols, rowptr, col.astype(np.int32))

    @staticmethod
    def from_dense(a: np.ndarray) -> "CSR":
        a = np.asarray(a, dtype=np.uint8) & 1
        return CSR.from_rows(a.shape[0], a.shape[1], [np.nonzero(r)[0] for r in a])

    def to_dense(self) -> np.ndarray:
        d = np.zeros((self.rows, self.cols), dtype=np.uint8)
        for r in range(self.rows):
            d[r, self.col[self.rowptr[r]:self.rowptr[r + 1]]] = 1
        return d

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def row(self, r: int) -> np.ndarray:
        return self.col[self.rowptr[r]:self.rowptr[r + 1]]

    def transpose(self) -> "CSR":
        lists = [[] for _ in range(self.cols)]
        for r in range(self.rows):
            for c in self.row(r):
                lists[c].append(r)
        return CSR.from_rows(self.cols, self.rows, lists)


@dataclass
class Code:
    """A CSS code seen from the decoder: X checks ``H`` and Z stabilisers ``G``.

    ``logicals`` optionally lists a basis of ker(G) modulo row(H) (one row
    per logical qubit) in closed form; without it the library finds one by
    GF(2) elimination.
    """

    name: str
    H: CSR
    G: CSR
    # sizes used in the literature's notation, kept for reporting only
    meta: dict = field(default_factory=dict)
    logicals: CSR | None = None

    @property
    def n(self) -> int:
        return self.H.cols

    @property
    def m(self) -> int:
        return self.H.rows


def _monomial_rows(l: int, m: int, terms, transpose: bool = False):
    """Row supports of the l*m x l*m matrix sum_k x^{a_k} y^{b_k}.

    Row ``i*m + j`` of ``x^a y^b`` has its single one in column
    ``((i + a) mod l)*m + (j + b) mod m`` (the shift ``S_k`` moves index i to
    i+1). ``transpose`` gives the rows of the transposed matrix.
    """
    out = []
    for i in range(l):
        for j in range(m):
            row = []
            for a, b in terms:
                if transpose:
                    row.append(((i - a) % l) * m + (j - b) % m)
                else:
                    row.append(((i + a) % l) * m + (j + b) % m)
            out.append(row)
    return out


def group_algebra_code(l: int, m: int, a_terms, b_terms, name: str) -> Code:
    """``H_X = [A | B]``, ``H_Z = [B^T | A^T]`` over ``F2[x,y]/(x^l - 1, y^m - 1)``.

    ``a_terms``/``b_terms`` list monomials ``x^a y^b`` as pairs ``(a, b)``.
    """
    N = l * m
    A = _monomial_rows(l, m, a_terms)
    B = _monomial_rows(l, m, b_terms)
    At = _monomial_rows(l, m, a_terms, transpose=True)
    Bt = _monomial_rows(l, m, b_terms, transpose=True)
    hx = [ra + [N + c for c in rb] for ra, rb in zip(A, B)]
    hz = [rb + [N + c for c in ra] for rb, ra in zip(Bt, At)]
    return Code(name, CSR.from_rows(N, 2 * N, hx), CSR.from_rows(N, 2 * N, hz),
                {"l": l, "m": m})


def toric_2d(L: int) -> Code:
    """2D toric code, ``A = 1 + x``, ``B = 1 + y``: n = 2L^2, m = L^2."""
    c = group_algebra_code(L, L, [(0, 0), (1, 0)], [(0, 0), (0, 1)], f"toric2d_L{L}")
    c.meta = {"L": L, "family": "toric2d"}
    # a row of A-block edges (a = 0, every b) and a column of B-block edges
    # (every a, b = 0): each meets every plaquette an even number of times
    c.logicals = CSR.from_rows(2, 2 * L * L, [[b for b in range(L)],
                                              [L * L + a * L for a in range(L)]])
    return c


def bivariate_bicycle(l: int, m: int) -> Code:
    """Bivariate-bicycle code with ``A = x^3 + y + y^2``, ``B = y^3 + x + x^2``."""
    c = group_algebra_code(l, m, [(3, 0), (0, 1), (0, 2)], [(0, 3), (1, 0), (2, 0)],
                           f"bb_{l}x{m}")
    c.meta = {"l": l, "m": m, "family": "bb"}
    return c


def _v3(L, x, y, z):
    return (x % L) + L * ((y % L) + L * (z % L))


def _toric3d_parts(L: int):
    L3 = L ** 3
    shift = [(1, 0, 0), (0, 1, 0), (0, 0, 1)]
    vertex_rows = []
    for z in range(L):
        for y in range(L):
            for x in range(L):
                v = _v3(L, x, y, z)
                row = []
                for a in range(3):
                    dx, dy, dz = shift[a]
                    row.append(a * L3 + v)  # e_a(v) starts at v
                    row.append(a * L3 + _v3(L, x - dx, y - dy, z - dz))  # e_a(v - a_hat) ends at v
                vertex_rows.append(row)
    face_rows = []
    for t, (a, b) in enumerate([(0, 1), (0, 2), (1, 2)]):
        for z in range(L):
            for y in range(L):
                for x in range(L):
                    v = _v3(L, x, y, z)
                    ax, ay, az = shift[a]
                    bx, by, bz = shift[b]
                    vb = _v3(L, x + bx, y + by, z + bz)
                    va = _v3(L, x + ax, y + ay, z + az)
                    face_rows.append([a * L3 + v, b * L3 + v, a * L3 + vb, b * L3 + va])
    return vertex_rows, face_rows


def toric_3d_point(L: int) -> Code:
    """3D toric code, point-like sector: vertex checks (weight 6), face stabilisers."""
    vr, fr = _toric3d_parts(L)
    L3 = L ** 3
    # edges of direction a crossing the plane v_a = 0 (L^2 each)
    logi = []
    for a in range(3):
        row = []
        for z in range(L):
            for y in range(L):
                for x in range(L):
                    if (x, y, z)[a] == 0:
                        row.append(a * L3 + _v3(L, x, y, z))
        logi.append(row)
    return Code(f"toric3d_point_L{L}", CSR.from_rows(L3, 3 * L3, vr),
                CSR.from_rows(3 * L3, 3 * L3, fr), {"L": L, "family": "toric3d_point"},
                CSR.from_rows(3, 3 * L3, logi))


def toric_3d_membrane(L: int) -> Code:
    """3D toric code, membrane-like sector: face checks (weight 4), vertex stabilisers."""
    vr, fr = _toric3d_parts(L)
    L3 = L ** 3
    # straight lines of direction a through the origin (L edges each)
    logi = []
    for a in range(3):
        row = []
        for t in range(L):
            xyz = [0, 0, 0]
            xyz[a] = t
            row.append(a * L3 + _v3(L, *xyz))
        logi.append(row)
    return Code(f"toric3d_membrane_L{L}", CSR.from_rows(3 * L3, 3 * L3, fr),
                CSR.from_rows(L3, 3 * L3, vr), {"L": L, "family": "toric3d_membrane"},
                CSR.from_rows(3, 3 * L3, logi))


def repetition(d: int, periodic: bool = True) -> Code:
    """Repetition code on d bits; periodic adds the check (d-1, 0)."""
    nchk = d if periodic else d - 1
    rows = [[j, (j + 1) % d] for j in range(nchk)]
    return Code(f"rep_d{d}{'_periodic' if periodic else '_open'}", CSR.from_rows(nchk, d, rows),
                CSR.from_rows(0, d, []), {"d": d, "family": "rep", "periodic": periodic})


def from_dense(H: np.ndarray, G: np.ndarray | None = None, name: str = "custom") -> Code:
    H = np.asarray(H, dtype=np.uint8)
    if G is None:
        G = np.zeros((0, H.shape[1]), dtype=np.uint8)
    return Code(name, CSR.from_dense(H), CSR.from_dense(G))


def by_name(name: str) -> Code:
    """Parse the names used in configs: ``toric2d:32``, ``toric3d_point:8``,
    ``toric3d_membrane:8``, ``bb:12x6``, ``rep:11``."""
    fam, _, arg = name.partition(":")
    if fam == "toric2d":
        return toric_2d(int(arg))
    if fam == "toric3d_point":
        return toric_3d_point(int(arg))
    if fam == "toric3d_membrane":
        return toric_3d_membrane(int(arg))
    if fam == "bb":
        l, m = arg.split("x")
        return bivariate_bicycle(int(l), int(m))
    if fam == "rep":
        return repetition(int(arg))
    raise ValueError(f"unknown code family {name!r}")
