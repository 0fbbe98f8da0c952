"""Oracle: H-LU factorisation with accumulated updates, plain FP64 numpy.

TEST INFRASTRUCTURE ONLY: the tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may use it; it shares no code with the GPU
library and never calls it.

What is computed.  A = L U without pivoting (Sec. 4.1) for an H-matrix A over
a binary cluster tree (Sec. 2.1, Definitions "Cluster Tree", "Block Tree"):
L unit lower triangular, U upper triangular, both with A's block structure
(a diagonal leaf holds the strict lower part of L and the upper part of U, as
a dense LU does).  The recursion is the block LU of the 2 x 2 structure:

    LU(A00);  A01 := L00^-1 A01;  A10 := A10 U00^-1;  A11 -= A10 A01;  LU(A11)

with the triangular solves recursing the same way (Sec. 2.2 states that
triangular solves and LU follow the pattern of the multiplication Alg. 2).

Updates go through accumulators and pending sets (Alg. 3, Sec. 2.2): each
block under work carries an accumulator (the sum of the updates evaluated so
far, dense for a dense leaf, low-rank otherwise) and a set of pending products
X_{t,r} Y_{r,s} (blocks of L and U that are already final).  On entering a
block, every product with a leaf factor is evaluated into its accumulator;
the others are split over the block's sons together with the restriction of
the accumulator.  A leaf evaluates all that is left, subtracts its
accumulator once, and then takes its own step: dense LU of a diagonal leaf,
a triangular solve of an off-diagonal one.

Low-rank sums are truncated by Alg. 1 (Sec. 2.2): QR of both factors, SVD of
R_U R_V^T, the smallest rank whose Frobenius tail of singular values is at
most eps times the whole.  With a storage format, a leaf of L or U is
compressed once it is final and every later read sees its decompressed
values (the semi-on-the-fly conversion of Alg. 4); accumulators stay FP64
(Sec. 4.1).

Readings where the paper is silent: an accumulator addition is a truncated
low-rank addition; a pending product with no leaf factor that reaches a leaf
is evaluated by the sons' products, assembled with zero padding into one
low-rank term and truncated; a dense term added to a low-rank accumulator is
first written as a low-rank product of rank min(rows, columns).
"""

from __future__ import annotations

import numpy as np
from scipy.linalg import solve_triangular

from .oracle import AFLP_BYTES, round_to


def trunc_rank(S: np.ndarray, eps: float) -> int:
    """Smallest k with (sum_{i >= k} S_i^2)^(1/2) <= eps (sum_i S_i^2)^(1/2)."""
    tot = float(np.sum(S * S))
    if tot == 0.0:
        return 0
    tail = np.concatenate([np.cumsum((S * S)[::-1])[::-1], [0.0]])   # tail[k] = sum_{i >= k}
    return int(np.flatnonzero(tail <= eps * eps * tot)[0])


def truncate(U: np.ndarray, V: np.ndarray, eps: float):
    """Alg. 1: U V^T ~ W X^T with W = Q_U U_s(:, :k) S_s(:k), X = Q_V V_s(:, :k)."""
    if U.shape[1] == 0:
        return U, V
    Qu, Ru = np.linalg.qr(U)
    Qv, Rv = np.linalg.qr(V)
    Us, S, Vst = np.linalg.svd(Ru @ Rv.T)
    k = trunc_rank(S, eps)
    return Qu @ (Us[:, :k] * S[:k]), Qv @ Vst[:k].T


def dense_of(term, m: int, n: int) -> np.ndarray:
    if term is None:
        return np.zeros((m, n))
    if term[0] == "D":
        return term[1]
    return term[1] @ term[2].T


def lowrank_of(term, m: int, n: int):
    """(U, V) of a term; a dense term of m x n as a product of rank min(m, n)."""
    if term is None:
        return np.zeros((m, 0)), np.zeros((n, 0))
    if term[0] == "R":
        return term[1], term[2]
    D = term[1]
    if m <= n:
        return np.eye(m), D.T.copy()
    return D.copy(), np.eye(n)


class HLU:
    """H-LU of the H-matrix ``H`` (an hmgen HMatrix with FP64 leaves) at
    truncation accuracy ``eps``; ``dt``: storage format of the final leaves
    (None: FP64).  ``factor()`` runs the factorisation in place; the leaves
    then hold L and U."""

    def __init__(self, H, eps: float, dt: int | None = None):
        tr = H.tree()
        self.beg, self.end = tr["begin"], tr["end"]
        self.sons = np.stack([tr["son0"], tr["son1"]], axis=1)
        if dt is not None and dt in AFLP_BYTES:
            raise ValueError("AFLP rounds per data block; give an elementwise format")
        self.eps, self.dt = eps, dt
        self.n = H.n
        self.leaf = {}
        for i in range(H.nblocks):
            a, b, s = H.factors(i)
            key = (int(tr["tau"][i]), int(tr["sigma"][i]))
            if not H.adm[i]:
                self.leaf[key] = ["D", np.array(a, dtype=np.float64)]
            else:
                U = np.array(a * s if s is not None else a, dtype=np.float64)
                self.leaf[key] = ["R", U, np.array(b, dtype=np.float64)]
        self.truncations = 0

    # -------------------------------------------------------------- structure
    def size(self, c: int) -> int:
        return int(self.end[c] - self.beg[c])

    def rel(self, c: int, parent: int) -> slice:
        """Rows of cluster c inside cluster parent."""
        a = int(self.beg[c] - self.beg[parent])
        return slice(a, a + self.size(c))

    def is_leaf(self, t: int, s: int) -> bool:
        return (t, s) in self.leaf

    # --------------------------------------------- block times dense (Sec. 2.1)
    def mul(self, t: int, s: int, Z: np.ndarray) -> np.ndarray:
        """block(t, s) @ Z."""
        B = self.leaf.get((t, s))
        if B is not None:
            return B[1] @ Z if B[0] == "D" else B[1] @ (B[2].T @ Z)
        out = np.zeros((self.size(t), Z.shape[1]))
        for ti in self.sons[t]:
            for sj in self.sons[s]:
                out[self.rel(ti, t)] += self.mul(ti, sj, Z[self.rel(sj, s)])
        return out

    def mul_t(self, t: int, s: int, Z: np.ndarray) -> np.ndarray:
        """block(t, s)^T @ Z."""
        B = self.leaf.get((t, s))
        if B is not None:
            return B[1].T @ Z if B[0] == "D" else B[2] @ (B[1].T @ Z)
        out = np.zeros((self.size(s), Z.shape[1]))
        for ti in self.sons[t]:
            for sj in self.sons[s]:
                out[self.rel(sj, s)] += self.mul_t(ti, sj, Z[self.rel(ti, t)])
        return out

    # ------------------------------------------ triangular solves, dense right sides
    def solve_lower(self, t: int, Z: np.ndarray) -> np.ndarray:
        """L_tt^-1 Z (L unit lower triangular)."""
        D = self.leaf.get((t, t))
        if D is not None:
            return solve_triangular(D[1], Z, lower=True, unit_diagonal=True)
        t0, t1 = self.sons[t]
        Z = Z.copy()
        r0, r1 = self.rel(t0, t), self.rel(t1, t)
        Z[r0] = self.solve_lower(t0, Z[r0])
        Z[r1] = self.solve_lower(t1, Z[r1] - self.mul(t1, t0, Z[r0]))
        return Z

    def solve_upper_t(self, s: int, Z: np.ndarray) -> np.ndarray:
        """U_ss^-T Z (so that (U_ss^-T Z)^T = Z^T U_ss^-1)."""
        D = self.leaf.get((s, s))
        if D is not None:
            return solve_triangular(D[1], Z, lower=False, trans="T")
        s0, s1 = self.sons[s]
        Z = Z.copy()
        r0, r1 = self.rel(s0, s), self.rel(s1, s)
        Z[r0] = self.solve_upper_t(s0, Z[r0])
        Z[r1] = self.solve_upper_t(s1, Z[r1] - self.mul_t(s0, s1, Z[r0]))
        return Z

    # ------------------------------------------------------ accumulator terms
    def add(self, acc, term, m: int, n: int, dense: bool):
        """acc + term: exact for a dense accumulator, truncated (Alg. 1) otherwise."""
        if dense:
            return ("D", dense_of(acc, m, n) + dense_of(term, m, n))
        Ua, Va = lowrank_of(acc, m, n)
        Ut, Vt = lowrank_of(term, m, n)
        self.truncations += 1
        W, X = truncate(np.hstack([Ua, Ut]), np.hstack([Va, Vt]), self.eps)
        return ("R", W, X)

    def product(self, t: int, r: int, s: int):
        """block(t, r) @ block(r, s) as a term over t x s."""
        X, Y = self.leaf.get((t, r)), self.leaf.get((r, s))
        if X is not None and X[0] == "R":                  # U (Y^T V)^T
            return ("R", X[1], self.mul_t(r, s, X[2]))
        if Y is not None and Y[0] == "R":                  # (X U) V^T
            return ("R", self.mul(t, r, Y[1]), Y[2])
        if X is not None:                                  # dense X: (Y^T X^T)^T
            return ("D", self.mul_t(r, s, X[1].T).T)
        if Y is not None:                                  # dense Y
            return ("D", self.mul(t, r, Y[1]))
        m, n = self.size(t), self.size(s)
        acc = None
        for ti in self.sons[t]:
            for sj in self.sons[s]:
                for rl in self.sons[r]:
                    U, V = lowrank_of(self.product(ti, rl, sj), self.size(ti), self.size(sj))
                    Up = np.zeros((m, U.shape[1]))
                    Vp = np.zeros((n, V.shape[1]))
                    Up[self.rel(ti, t)] = U
                    Vp[self.rel(sj, s)] = V
                    acc = self.add(acc, ("R", Up, Vp), m, n, False)
        return acc

    def dense_target(self, t: int, s: int) -> bool:
        B = self.leaf.get((t, s))
        return B is not None and B[0] == "D"

    def gather(self, t: int, s: int, acc, pend: list):
        """Evaluate the pending products of block (t, s) that have a leaf
        factor (at a leaf: all of them) into its accumulator; return the
        accumulator and the products left pending."""
        m, n = self.size(t), self.size(s)
        at_leaf = self.is_leaf(t, s)
        dense = self.dense_target(t, s)
        rest = []
        for (a, r, b) in pend:
            if at_leaf or self.is_leaf(a, r) or self.is_leaf(r, b):
                acc = self.add(acc, self.product(a, r, b), m, n, dense)
            else:
                rest.append((a, r, b))
        return acc, rest

    def split(self, t: int, s: int, acc, pend: list) -> dict:
        """Accumulator and pending products of the four sons of block (t, s)."""
        out = {}
        for i, ti in enumerate(self.sons[t]):
            for j, sj in enumerate(self.sons[s]):
                if acc is None:
                    a = None
                else:
                    U, V = acc[1], acc[2]
                    a = ("R", U[self.rel(ti, t)], V[self.rel(sj, s)])
                    if self.dense_target(ti, sj):
                        a = ("D", a[1] @ a[2].T)
                p = [(ti, rl, sj) for (_, r, _) in pend for rl in self.sons[r]]
                out[i, j] = [a, p]
        return out

    def apply(self, t: int, s: int, acc) -> None:
        """Leaf (t, s) -= its accumulator."""
        if acc is None:
            return
        B = self.leaf[(t, s)]
        if B[0] == "D":
            B[1] = B[1] - dense_of(acc, self.size(t), self.size(s))
        else:
            Ua, Va = lowrank_of(acc, self.size(t), self.size(s))
            self.truncations += 1
            B[1], B[2] = truncate(np.hstack([B[1], -Ua]), np.hstack([B[2], Va]), self.eps)

    def finalize(self, t: int, s: int) -> None:
        """Compress a final leaf (its decompressed values replace it)."""
        if self.dt is None:
            return
        B = self.leaf[(t, s)]
        for q in range(1, len(B)):
            B[q] = round_to(B[q].reshape(-1, order="F"), self.dt).reshape(B[q].shape, order="F")

    # ----------------------------------------------------------- the recursion
    def lu(self, t: int, acc=None, pend=None) -> None:
        acc, pend = self.gather(t, t, acc, pend or [])
        if self.is_leaf(t, t):
            self.apply(t, t, acc)
            D = self.leaf[(t, t)][1]
            for k in range(D.shape[0] - 1):                # dense LU, no pivoting
                D[k + 1:, k] /= D[k, k]
                D[k + 1:, k + 1:] -= np.outer(D[k + 1:, k], D[k, k + 1:])
            self.finalize(t, t)
            return
        t0, t1 = self.sons[t]
        sub = self.split(t, t, acc, pend)
        self.lu(t0, *sub[0, 0])
        self.solve_l(t0, t1, *sub[0, 1])                   # U01 = L00^-1 A01
        self.solve_u(t1, t0, *sub[1, 0])                   # L10 = A10 U00^-1
        sub[1, 1][1].append((t1, t0, t1))                  # A11 -= L10 U01
        self.lu(t1, *sub[1, 1])

    def solve_l(self, t: int, s: int, acc=None, pend=None) -> None:
        """block(t, s) := L_tt^-1 (block(t, s) - updates)."""
        acc, pend = self.gather(t, s, acc, pend or [])
        if self.is_leaf(t, s):
            self.apply(t, s, acc)
            B = self.leaf[(t, s)]
            B[1] = self.solve_lower(t, B[1])               # D, or U of U V^T
            self.finalize(t, s)
            return
        t0, t1 = self.sons[t]
        sub = self.split(t, s, acc, pend)
        for j, sj in enumerate(self.sons[s]):
            self.solve_l(t0, sj, *sub[0, j])
            sub[1, j][1].append((t1, t0, sj))              # B1j -= L10 X0j
            self.solve_l(t1, sj, *sub[1, j])

    def solve_u(self, t: int, s: int, acc=None, pend=None) -> None:
        """block(t, s) := (block(t, s) - updates) U_ss^-1."""
        acc, pend = self.gather(t, s, acc, pend or [])
        if self.is_leaf(t, s):
            self.apply(t, s, acc)
            B = self.leaf[(t, s)]
            if B[0] == "D":
                B[1] = self.solve_upper_t(s, B[1].T).T
            else:
                B[2] = self.solve_upper_t(s, B[2])         # V of U V^T
            self.finalize(t, s)
            return
        s0, s1 = self.sons[s]
        sub = self.split(t, s, acc, pend)
        for i, ti in enumerate(self.sons[t]):
            self.solve_u(ti, s0, *sub[i, 0])
            sub[i, 1][1].append((ti, s0, s1))              # Bi1 -= Xi0 U01
            self.solve_u(ti, s1, *sub[i, 1])

    def factor(self) -> "HLU":
        self.lu(0)
        return self

    # -------------------------------------------------------------- results
    def solve(self, b: np.ndarray) -> np.ndarray:
        """(L U)^-1 b (cluster order), by the two H-triangular solves."""
        z = self.solve_lower(0, np.asarray(b, dtype=np.float64).reshape(self.n, -1))
        return self.solve_upper(0, z)

    def solve_upper(self, s: int, Z: np.ndarray) -> np.ndarray:
        """U_ss^-1 Z."""
        D = self.leaf.get((s, s))
        if D is not None:
            return solve_triangular(D[1], Z, lower=False)
        s0, s1 = self.sons[s]
        Z = Z.copy()
        r0, r1 = self.rel(s0, s), self.rel(s1, s)
        Z[r1] = self.solve_upper(s1, Z[r1])
        Z[r0] = self.solve_upper(s0, Z[r0] - self.mul(s0, s1, Z[r1]))
        return Z

    def assemble(self):
        """Dense L and U (cluster order)."""
        L = np.eye(self.n)
        U = np.zeros((self.n, self.n))
        for (t, s), B in self.leaf.items():
            r = slice(int(self.beg[t]), int(self.end[t]))
            c = slice(int(self.beg[s]), int(self.end[s]))
            M = dense_of(tuple(B), self.size(t), self.size(s))
            if t == s:
                L[r, c] += np.tril(M, -1)
                U[r, c] = np.triu(M)
            elif self.beg[t] > self.beg[s]:
                L[r, c] = M
            else:
                U[r, c] = M
        return L, U

    def leaf_matrix(self, t: int, s: int) -> np.ndarray:
        return dense_of(tuple(self.leaf[(t, s)]), self.size(t), self.size(s))


def assemble_h(H) -> np.ndarray:
    """The dense matrix of an H-matrix (cluster order)."""
    A = np.zeros((H.n, H.n))
    for i in range(H.nblocks):
        a, b, s = H.factors(i)
        if not H.adm[i]:
            M = a
        else:
            M = (a * s) @ b.T if s is not None else a @ b.T
        A[H.rb[i]:H.re[i], H.cb[i]:H.ce[i]] = M
    return A


def lu_error(A: np.ndarray, L: np.ndarray, U: np.ndarray) -> float:
    """|| I - A (L U)^-1 ||_2 (Sec. 4.1), dense."""
    n = A.shape[0]
    inv = solve_triangular(U, solve_triangular(L, np.eye(n), lower=True, unit_diagonal=True), lower=False)
    return float(np.linalg.norm(np.eye(n) - A @ inv, 2))
