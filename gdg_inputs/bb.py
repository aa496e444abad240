"""Bivariate-bicycle (BB) codes and GF(2) linear algebra.

Input generation only: this module builds the parity-check matrices the decoder
is run on. It holds none of the decoder's arithmetic and is shared, as an input
generator, by the GPU path's tests and by the CPU oracle.

Construction (Appendix B, the N=288 syndrome-code discussion): H_X = [A|B] with
x = S_l (x) I_m, y = I_l (x) S_m, S the cyclic shift matrix, and a monomial
x^a y^b placed at index m*a + b. H_Z = [B^T | A^T] is the matching Z-check
matrix of the bicycle construction (the same appendix uses H_Z and H_X^perp).
The shift convention is S[i, (i+1) mod l] = 1; it is pinned by the appendix's
statement that, for N=288, the first columns of A and B are y^5+y^10+x^9 and
y^9+x^10+x^11.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


def shift_matrix(n: int) -> np.ndarray:
    s = np.zeros((n, n), dtype=np.uint8)
    for i in range(n):
        s[i, (i + 1) % n] = 1
    return s


def monomial(l: int, m: int, a: int, b: int) -> np.ndarray:
    """Matrix of x^a y^b, x = S_l (x) I_m, y = I_l (x) S_m."""
    x = np.kron(shift_matrix(l), np.eye(m, dtype=np.uint8))
    y = np.kron(np.eye(l, dtype=np.uint8), shift_matrix(m))
    out = np.eye(l * m, dtype=np.int64)
    for _ in range(a % l):
        out = out @ x
    for _ in range(b % m):
        out = out @ y
    return (out % 2).astype(np.uint8)


def poly_matrix(l: int, m: int, terms) -> np.ndarray:
    """Sum (mod 2) of monomials; terms is a list of (a, b) exponent pairs."""
    out = np.zeros((l * m, l * m), dtype=np.uint8)
    for a, b in terms:
        out ^= monomial(l, m, a, b)
    return out


# ---------------------------------------------------------------- GF(2) algebra

def gf2_rref(mat: np.ndarray):
    """Row-reduce a 0/1 matrix over GF(2). Returns (rref, pivot_columns)."""
    a = (np.array(mat, dtype=np.uint8) & 1).copy()
    rows, cols = a.shape
    piv = []
    r = 0
    for c in range(cols):
        if r >= rows:
            break
        nz = np.nonzero(a[r:, c])[0]
        if nz.size == 0:
            continue
        p = r + nz[0]
        if p != r:
            a[[r, p]] = a[[p, r]]
        hit = np.nonzero(a[:, c])[0]
        hit = hit[hit != r]
        if hit.size:
            a[hit] ^= a[r]
        piv.append(c)
        r += 1
    return a, piv


def gf2_rank(mat: np.ndarray) -> int:
    return len(gf2_rref(mat)[1])


def gf2_nullspace(mat: np.ndarray) -> np.ndarray:
    """Basis (as rows) of {v : mat v = 0} over GF(2)."""
    mat = np.array(mat, dtype=np.uint8) & 1
    rows, cols = mat.shape
    rref, piv = gf2_rref(mat)
    free = [c for c in range(cols) if c not in set(piv)]
    basis = []
    for f in free:
        v = np.zeros(cols, dtype=np.uint8)
        v[f] = 1
        for i, pc in enumerate(piv):
            if rref[i, f]:
                v[pc] = 1
        basis.append(v)
    if not basis:
        return np.zeros((0, cols), dtype=np.uint8)
    return np.array(basis, dtype=np.uint8)


def logical_operators(h_check: np.ndarray, h_other: np.ndarray) -> np.ndarray:
    """Logical operators that detect the errors h_check sees.

    An error e is seen through its syndrome h_check e. A logical operator that
    detects such errors is an operator of the check type of h_check that
    commutes with every stabiliser in h_other, i.e. a vector of ker(h_other),
    and is not itself a stabiliser, i.e. independent of rowspace(h_check).
    Returns K = dim ker(h_other) - rank(h_check) such rows.
    """
    ker = gf2_nullspace(h_other)
    base = np.array(h_check, dtype=np.uint8) & 1
    r0 = gf2_rank(base)
    chosen = []
    cur = base
    cur_rank = r0
    for v in ker:
        trial = np.vstack([cur, v[None, :]])
        rk = gf2_rank(trial)
        if rk > cur_rank:
            chosen.append(v)
            cur = trial
            cur_rank = rk
    return np.array(chosen, dtype=np.uint8)


# ---------------------------------------------------------------- BB codes

@dataclass
class BBCode:
    name: str
    l: int
    m: int
    a_terms: list
    b_terms: list
    hx: np.ndarray = field(repr=False, default=None)
    hz: np.ndarray = field(repr=False, default=None)
    a: np.ndarray = field(repr=False, default=None)
    b: np.ndarray = field(repr=False, default=None)

    @property
    def n(self) -> int:
        return 2 * self.l * self.m

    @property
    def w(self) -> int:
        """Checks of one type, N/2."""
        return self.l * self.m

    def k(self) -> int:
        return self.n - gf2_rank(self.hx) - gf2_rank(self.hz)


def bb_code(name, l, m, a_terms, b_terms) -> BBCode:
    a = poly_matrix(l, m, a_terms)
    b = poly_matrix(l, m, b_terms)
    hx = np.hstack([a, b])
    hz = np.hstack([b.T, a.T])
    return BBCode(name, l, m, list(a_terms), list(b_terms), hx, hz, a, b)


# Polynomials as lists of (x exponent, y exponent).
_X3_Y_Y2 = [(3, 0), (0, 1), (0, 2)]
_Y3_X_X2 = [(0, 3), (1, 0), (2, 0)]

CODES = {
    "72": dict(name="[[72,12,6]]", l=6, m=6, a_terms=_X3_Y_Y2, b_terms=_Y3_X_X2),
    "90": dict(name="[[90,8,10]]", l=15, m=3, a_terms=[(9, 0), (0, 1), (0, 2)],
               b_terms=[(0, 0), (2, 0), (7, 0)]),
    "108": dict(name="[[108,8,10]]", l=9, m=6, a_terms=_X3_Y_Y2, b_terms=_Y3_X_X2),
    "144": dict(name="[[144,12,12]]", l=12, m=6, a_terms=_X3_Y_Y2, b_terms=_Y3_X_X2),
    "288": dict(name="[[288,12,18]]", l=12, m=12, a_terms=[(3, 0), (0, 2), (0, 7)],
                b_terms=[(0, 3), (1, 0), (2, 0)]),
}

CODE_K = {"72": 12, "90": 8, "108": 8, "144": 12, "288": 12}
CODE_D = {"72": 6, "90": 10, "108": 10, "144": 12, "288": 18}


def get_code(key: str) -> BBCode:
    return bb_code(**CODES[str(key)])
