"""Independent full-space constructions used to pin the oracle.

Nothing here is shared with the oracle or the GPU library: dense operators
are built from Pauli matrices with Kronecker products, the group acts on the
full 2^N space by permuting basis vectors (vectorised numpy), and sector
bases come from the projector P = (1/|G|) sum_g conj(chi(g)) U_g.
"""
from __future__ import annotations

from math import comb

import numpy as np

SX = np.array([[0, 1], [1, 0]], dtype=np.complex128)
SY = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
SZ = np.array([[1, 0], [0, -1]], dtype=np.complex128)   # |up> = bit 1 first below


def site_op(op: np.ndarray, i: int, n: int) -> np.ndarray:
    """op acting on site i of n; basis index = bitstring with bit i = site i,
    bit value 1 = up.  Built as a kron product over sites n-1 ... 0."""
    # local basis order (bit=0, bit=1) = (down, up); convert op from (up, down)
    P = np.array([[0, 1], [1, 0]])
    loc = P @ op @ P
    out = np.array([[1.0 + 0j]])
    for k in range(n - 1, -1, -1):
        out = np.kron(out, loc if k == i else np.eye(2))
    return out


def heisenberg_full(n: int, bonds) -> np.ndarray:
    H = np.zeros((2 ** n, 2 ** n), dtype=np.complex128)
    ops = {}
    for a in (SX, SY, SZ):
        for i in range(n):
            ops[(id(a), i)] = site_op(a, i, n)
    for i, j, J in bonds:
        for a in (SX, SY, SZ):
            H += (J / 4.0) * ops[(id(a), i)] @ ops[(id(a), j)]
    return H


def group_action_matrix(n: int, perm, flip) -> np.ndarray:
    """U_g on the full space: |s> -> |g.s>, bit i of s to bit perm[i]."""
    s = np.arange(2 ** n, dtype=np.int64)
    t = np.zeros_like(s)
    for i in range(n):
        t |= ((s >> i) & 1) << int(perm[i])
    if flip:
        t ^= (1 << n) - 1
    U = np.zeros((2 ** n, 2 ** n))
    U[t, s] = 1.0
    return U


def projector(n: int, group) -> np.ndarray:
    P = np.zeros((2 ** n, 2 ** n), dtype=np.complex128)
    chi = group.chi[:, 0] + 1j * group.chi[:, 1]
    for g in range(group.size):
        P += np.conj(chi[g]) * group_action_matrix(n, group.perm[g], group.flip[g])
    return P / group.size


def sector_basis(n: int, weight: int, group, reps) -> np.ndarray:
    """Columns P|r>/||P|r>|| for the given representatives."""
    P = projector(n, group)
    B = np.zeros((2 ** n, len(reps)), dtype=np.complex128)
    for k, r in enumerate(reps):
        v = P[:, int(r)]
        B[:, k] = v / np.linalg.norm(v)
    return B


def weight_states(n: int, w: int) -> np.ndarray:
    s = np.arange(2 ** n, dtype=np.int64)
    pc = np.array([bin(int(v)).count("1") for v in s])
    return s[pc == w] if w >= 0 else s


def cycles(perm) -> list:
    n = len(perm)
    seen = [False] * n
    out = []
    for i in range(n):
        if not seen[i]:
            L = 0
            j = i
            while not seen[j]:
                seen[j] = True
                j = int(perm[j])
                L += 1
            out.append(L)
    return out


def fixed_count(perm, flip, n: int, w: int) -> int:
    """Number of states of weight w (any weight if w < 0) fixed by (perm, flip)."""
    cyc = cycles(perm)
    if flip:
        if any(L % 2 for L in cyc):
            return 0
        if w >= 0 and 2 * w != n:
            return 0
        return 2 ** len(cyc)
    if w < 0:
        return 2 ** len(cyc)
    poly = [1]
    for L in cyc:
        new = [0] * (len(poly) + L)
        for k, c in enumerate(poly):
            new[k] += c
            new[k + L] += c
        poly = new
    return poly[w] if w < len(poly) else 0


def character_dimension(group, w: int) -> int:
    """dim = (1/|G|) sum_g conj(chi(g)) fix_w(g) (Burnside/character formula)."""
    chi = group.chi[:, 0] + 1j * group.chi[:, 1]
    tot = 0j
    for g in range(group.size):
        tot += np.conj(chi[g]) * fixed_count(group.perm[g], group.flip[g], group.n_sites, w)
    val = tot / group.size
    d = int(round(val.real))
    assert abs(val - d) < 1e-6, val
    return d


def colex_rank(s: int) -> int:
    """Position of s among all bitstrings of its weight in increasing order:
    sum over set bits p_0 < p_1 < ... of C(p_k, k+1)."""
    r, k, p = 0, 0, 0
    while s:
        if s & 1:
            r += comb(p, k + 1)
            k += 1
        s >>= 1
        p += 1
    return r


def bethe_ground_energy(n: int, J: float = 1.0) -> float:
    """Ground energy of the closed spin-1/2 Heisenberg chain H = J sum_i
    S_i . S_{i+1} (J > 0, even n) from Bethe's ansatz: M = n/2 magnons with
    rapidities lambda_j solving the logarithmic Bethe equations
        n * 2 atan(2 lambda_j) = 2 pi I_j + sum_{k != j} 2 atan(lambda_j - lambda_k),
    I_j = -(M-1)/2, ..., (M-1)/2 (the ground state's quantum numbers), and
        E = J n / 4 - sum_j (J/2) / (lambda_j^2 + 1/4).
    Solved by the standard fixed-point iteration lambda_j = tan(...)/2,
    then Newton's method on the equations above to machine precision."""
    if n % 2 or n < 2:
        raise ValueError("even n >= 2")
    M = n // 2
    I = -(M - 1) / 2.0 + np.arange(M)
    lam = 0.5 * np.tan(np.pi * I / n)
    for _ in range(5000):
        d = lam[:, None] - lam[None, :]
        new = 0.5 * np.tan((np.pi * I + np.arctan(d).sum(axis=1)) / n)
        done = np.max(np.abs(new - lam)) < 1e-15
        lam = new
        if done:
            break
    for _ in range(100):
        d = lam[:, None] - lam[None, :]
        F = 2 * n * np.arctan(2 * lam) - 2 * np.pi * I - 2 * np.arctan(d).sum(axis=1)
        Jm = 2.0 / (1.0 + d ** 2)
        np.fill_diagonal(Jm, 0.0)
        diag = 4 * n / (1 + 4 * lam ** 2) - Jm.sum(axis=1)
        np.fill_diagonal(Jm, diag)
        step = np.linalg.solve(Jm, -F)
        lam = lam + step
        if np.max(np.abs(step)) < 1e-15:
            break
    return float(J * n / 4.0 - J * np.sum(0.5 / (lam ** 2 + 0.25)))
