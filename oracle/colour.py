"""Colour algebra for the oracle, from explicit Gell-Mann matrices (numpy, FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

* ``colour_matrix(m)``: the matrix of the colour quadratic form that aggregates
  colour-ordered partial amplitudes into |M|^2 (the "aggregate their
  contribution" step of Sec. 2.2), for a quark line with m gluons:
  C[s, s'] = sum over adjoint indices of Tr((t^{s_1}...t^{s_m})^dagger t^{s'_1}...t^{s'_m}),
  orderings s in lexicographic order, t^a = lambda^a / 2.
* ``dressed_me(m, mom, mt)``: |M|^2 summed over all explicit colours and
  helicities by a colour-dressed Berends-Giele recursion that uses the full QCD
  Feynman rules (structure constants f^{abc}, generators t^a) instead of the
  colour decomposition -- an independent route to the same number, used only
  to pin the colour-ordered recursion of the oracle on small multiplicities.
"""
from __future__ import annotations

import functools
import itertools

import numpy as np


def generators() -> np.ndarray:
    """t^a = lambda^a / 2 (Gell-Mann), shape (8, 3, 3)."""
    l = np.zeros((8, 3, 3), dtype=np.complex128)
    l[0][0, 1] = l[0][1, 0] = 1
    l[1][0, 1] = -1j
    l[1][1, 0] = 1j
    l[2][0, 0] = 1
    l[2][1, 1] = -1
    l[3][0, 2] = l[3][2, 0] = 1
    l[4][0, 2] = -1j
    l[4][2, 0] = 1j
    l[5][1, 2] = l[5][2, 1] = 1
    l[6][1, 2] = -1j
    l[6][2, 1] = 1j
    l[7][0, 0] = l[7][1, 1] = 1 / np.sqrt(3)
    l[7][2, 2] = -2 / np.sqrt(3)
    return l / 2


def structure_constants() -> np.ndarray:
    """f^{abc} from [t^a, t^b] = i f^{abc} t^c, i.e. f^{abc} = -2i Tr([t^a,t^b] t^c)."""
    t = generators()
    comm = np.einsum("aij,bjk->abik", t, t, optimize=True) - np.einsum("bij,ajk->abik", t, t, optimize=True)
    f = -2j * np.einsum("abij,cji->abc", comm, t, optimize=True)
    assert np.max(np.abs(f.imag)) < 1e-12
    return f.real


def _words(m: int, order) -> np.ndarray:
    """t^{a_{order[0]}} ... t^{a_{order[m-1]}} for every assignment a, shape (8,)*m + (3,3)."""
    t = generators()
    W = np.eye(3, dtype=np.complex128).reshape((1,) * m + (3, 3))
    for g in order:
        shape = [1] * m + [3, 3]
        shape[g] = 8
        W = W @ t.reshape(shape)
    return W


def _trace_pair(m: int, s, sp) -> float:
    A = _words(m, s)
    B = _words(m, sp)
    return float(np.sum(np.conj(A) * B).real)


@functools.lru_cache(maxsize=None)
def colour_matrix(m: int) -> np.ndarray:
    perms = list(itertools.permutations(range(m)))
    nf = len(perms)
    if m <= 4:
        W = np.stack([_words(m, p).reshape(-1) for p in perms])  # (nf, 8^m * 9)
        C = (np.conj(W) @ W.T).real
        return np.ascontiguousarray(C)
    # m = 5: relabelling the summed adjoint indices by s gives
    # C[s, s'] = C[id, pi] with pi_k = s^{-1}(s'_k); the first row is summed
    # explicitly (the identity is checked against the full sum for m <= 4).
    W0 = np.conj(_words(m, perms[0]))
    row = np.array([float(np.sum(W0 * _words(m, p)).real) for p in perms])
    index = {p: i for i, p in enumerate(perms)}
    C = np.zeros((nf, nf))
    for i, s in enumerate(perms):
        inv = np.argsort(s)
        for j, sp in enumerate(perms):
            pi = tuple(int(inv[x]) for x in sp)
            C[i, j] = row[index[pi]]
    return C


def colour_matrix_by_relabelling(m: int) -> np.ndarray:
    """Same as colour_matrix(5)'s construction, for any m (used to test the identity)."""
    perms = list(itertools.permutations(range(m)))
    W0 = np.conj(_words(m, perms[0]))
    row = np.array([float(np.sum(W0 * _words(m, p)).real) for p in perms])
    index = {p: i for i, p in enumerate(perms)}
    C = np.zeros((len(perms), len(perms)))
    for i, s in enumerate(perms):
        inv = np.argsort(s)
        for j, sp in enumerate(perms):
            C[i, j] = row[index[tuple(int(inv[x]) for x in sp)]]
    return C


# ----------------------------------------------------------- explicit colour
_METRIC = np.array([1.0, -1.0, -1.0, -1.0])


def _mdot(a, b):
    """Minkowski product over the last axis (no conjugation)."""
    return a[..., 0] * b[..., 0] - a[..., 1] * b[..., 1] - a[..., 2] * b[..., 2] - a[..., 3] * b[..., 3]


def dressed_me(m: int, mom: np.ndarray, mt: float, helicities=None):
    """Colour- and helicity-summed |M|^2 (g = 1) for g g -> t t~ + (m-2) g with explicit colours.

    mom = (p1, p2, top, antitop, gluons...) physical momenta, p1 and p2 incoming.
    Feynman rules (metric +---, Feynman gauge, all vertex momenta incoming):
    quark-gluon i g gamma^mu t^a; three-gluon g f^{abc}[g^{mu nu}(k-p)^rho +
    g^{nu rho}(p-q)^mu + g^{rho mu}(q-k)^nu]; four-gluon -i g^2 [f^{abe}f^{cde}
    (g^{mu rho}g^{nu sigma} - g^{mu sigma}g^{nu rho}) + (b<->c) + (b<->d)
    arrangements]; propagators -i g_{mu nu}/k^2 and i(pslash+m)/(p^2-m^2).
    With ``helicities`` (indices in the oracle's helicity numbering) the
    per-helicity colour sums are returned instead of the total.
    """
    from . import gamma_matrices, wavefunction

    mom = np.asarray(mom, dtype=np.float64)
    G = gamma_matrices()  # [mu][r][c]
    t = generators()
    f = structure_constants()
    FF1 = np.einsum("abe,cde->abcd", f, f, optimize=True)
    FF2 = np.einsum("ace,bde->abcd", f, f, optimize=True)
    FF3 = np.einsum("ade,bce->abcd", f, f, optimize=True)
    kph = [mom[0], mom[1]] + [mom[4 + i] for i in range(m - 2)]
    incoming = [True, True] + [False] * (m - 2)
    kout = [(-k if inc else k) for k, inc in zip(kph, incoming)]
    pt, ptb = mom[2], mom[3]
    B = 8**m
    digits = np.array(list(itertools.product(range(8), repeat=m)))  # (B, m), gluon i colour = digits[:, i]
    full = (1 << m) - 1

    def P(S):
        return sum(kout[i] for i in range(m) if S >> i & 1)

    def slash_b(J):  # J (..., 4) contravariant -> (..., 4, 4)
        return np.einsum("m,mrc,...m->...rc", _METRIC, G, J, optimize=True)

    total = 0.0
    per = []
    for h in (range(1 << (m + 2)) if helicities is None else helicities):
        lam = [1 if (h >> (m + 1 - i)) & 1 else -1 for i in range(m)]
        lt = 1 if (h >> 1) & 1 else -1
        ltb = 1 if h & 1 else -1
        eps = [wavefunction("eps" if incoming[i] else "eps*", kph[i], 0.0, lam[i]) for i in range(m)]
        ubar = wavefunction("ubar", pt, mt, lt)
        v = wavefunction("v", ptb, mt, ltb)
        J = {}
        for i in range(m):
            a = np.zeros((B, 8, 4), dtype=np.complex128)
            a[np.arange(B), digits[:, i], :] = eps[i]
            J[1 << i] = a
        for S in sorted(range(1, full + 1), key=lambda s: bin(s).count("1")):
            if bin(S).count("1") < 2:
                continue
            low = S & -S
            V = np.zeros((B, 8, 4), dtype=np.complex128)
            sub = (S - 1) & S
            while sub:
                S1, S2 = sub, S ^ sub
                if S1 & low and S2:
                    J1, J2 = J[S1], J[S2]
                    k = P(S)
                    p = -P(S1)
                    q = -P(S2)
                    kp = _mdot(J2, (k - p)[None, None, :])          # (B, c)
                    qk = _mdot(J1, (q - k)[None, None, :])          # (B, b)
                    d12 = np.einsum("Bbm,Bcm,m->Bbc", J1, J2, _METRIC, optimize=True)
                    V += np.einsum("abc,Bbm,Bc->Bam", f, J1, kp, optimize=True)
                    V += np.einsum("abc,Bbc->Ba", f, d12, optimize=True)[:, :, None] * (p - q)[None, None, :]
                    V += np.einsum("abc,Bcm,Bb->Bam", f, J2, qk, optimize=True)
                sub = (sub - 1) & S
            # four-gluon vertex: unordered triples
            sub = (S - 1) & S
            while sub:
                S1 = sub
                if S1 & low:
                    rest = S ^ S1
                    low2 = rest & -rest if rest else 0
                    sub2 = (rest - 1) & rest if rest else 0
                    while sub2:
                        S2, S3 = sub2, rest ^ sub2
                        if S2 & low2 and S3:
                            J1, J2, J3 = J[S1], J[S2], J[S3]
                            d13 = np.einsum("Bbm,Bdm,m->Bbd", J1, J3, _METRIC, optimize=True)
                            d12 = np.einsum("Bbm,Bcm,m->Bbc", J1, J2, _METRIC, optimize=True)
                            d23 = np.einsum("Bcm,Bdm,m->Bcd", J2, J3, _METRIC, optimize=True)
                            W = np.einsum("abcd,Bcm,Bbd->Bam", FF1, J2, d13, optimize=True)
                            W -= np.einsum("abcd,Bdm,Bbc->Bam", FF1, J3, d12, optimize=True)
                            W += np.einsum("abcd,Bbm,Bcd->Bam", FF2, J1, d23, optimize=True)
                            W -= np.einsum("abcd,Bdm,Bbc->Bam", FF2, J3, d12, optimize=True)
                            W += np.einsum("abcd,Bbm,Bcd->Bam", FF3, J1, d23, optimize=True)
                            W -= np.einsum("abcd,Bcm,Bbd->Bam", FF3, J2, d13, optimize=True)
                            V += -1j * W
                        sub2 = (sub2 - 1) & rest
                sub = (sub - 1) & S
            PS = P(S)
            J[S] = (-1j / _mdot(PS, PS)) * V
        # quark line: Psi[S] (B, k, j, 4)
        Psi = {0: np.einsum("kj,r->kjr", np.eye(3), v, optimize=True)[None].repeat(B, axis=0)}

        def attach(S):
            acc = np.zeros((B, 3, 3, 4), dtype=np.complex128)
            sub = S
            while sub:
                S1 = sub
                rest = S ^ S1
                if rest in Psi:
                    sl = slash_b(J[S1])  # (B, a, r, c)
                    acc += 1j * np.einsum("akl,Barc,Bljc->Bkjr", t, sl, Psi[rest], optimize=True)
                sub = (sub - 1) & S
            return acc

        for S in sorted(range(1, full), key=lambda s: bin(s).count("1")):
            p = -ptb - P(S)
            ps = np.einsum("m,mrc,m->rc", _METRIC, G, p, optimize=True) + mt * np.eye(4)
            Psi[S] = (1j / (_mdot(p, p) - mt * mt)) * np.einsum("rs,Bkjs->Bkjr", ps, attach(S), optimize=True)
        amp = np.einsum("r,Bijr->Bij", ubar, attach(full), optimize=True)
        per.append(float(np.sum(np.abs(amp) ** 2)))
        total += per[-1]
    return total if helicities is None else np.array(per)


@functools.lru_cache(maxsize=None)
def two_line_colour_tensors() -> np.ndarray:
    """Colour tensors C_d[a, L_row, L_col, T_row, T_col] of the five diagrams of
    a light quark line and the top line joined by one gluon, with one more
    external gluon of adjoint index a (see oracle.cpp, two quark lines):
      d = 0: (t^b t^a)_L (t^b)_T     d = 1: (t^a t^b)_L (t^b)_T
      d = 2: (t^c)_L (t^a t^c)_T     d = 3: (t^c)_L (t^c t^a)_T
      d = 4: f^{abc} (t^b)_L (t^c)_T
    summed over the internal adjoint indices, shape (5, 8, 3, 3, 3, 3)."""
    t = generators()
    f = structure_constants()
    C = np.zeros((5, 8, 3, 3, 3, 3), dtype=np.complex128)
    C[0] = np.einsum("bij,ajk,blm->aiklm", t, t, t)
    C[1] = np.einsum("aij,bjk,blm->aiklm", t, t, t)
    C[2] = np.einsum("cik,alj,cjm->aiklm", t, t, t)
    C[3] = np.einsum("cik,clj,ajm->aiklm", t, t, t)
    C[4] = np.einsum("abc,bik,clm->aiklm", f, t, t)
    return C


@functools.lru_cache(maxsize=None)
def two_line_colour_matrix() -> np.ndarray:
    """CC[d, d'] = sum over every colour index of C_d C_d'^* (complex 5 x 5)."""
    C = two_line_colour_tensors().reshape(5, -1)
    return np.ascontiguousarray(C @ np.conj(C).T)
