"""Build-time generator of the per-process amplitude code (HIP, gfx950).

For g g -> t t~ + (m-2) g it writes one header ``me_gg_m{m}.h`` holding a
device function that returns the colour- and polarisation-summed |M|^2
(coupling set to 1) of one event, as straight-line code:

* all momenta outgoing; gluon currents for every ordered sequence of gluons,
  built from the colour-ordered three- and four-gluon vertices (Berends-Giele
  recursion, the off-shell "_1/_2/_3" vertex forms of Sec. 2.2);
* the top line from the antitop end: Psi(seq) = prop(seq) * sum_j
  slash(J(seq_1..j)) Psi(seq_j+1..), closed with ubar(top) into the
  colour-ordered partial amplitudes A(sigma);
* the colour quadratic form sum_{s,s'} A_s^* C_{ss'} A_s' with the exact
  rational colour matrix, grouped by its distinct entries.

Gluons use real linear polarisation vectors, so every pure-gluon current is
a real four-vector; the top spinors are helicity eigenstates.  The sum over
the two linear polarisations equals the sum over helicities exactly.

The colour matrix C[s][s'] = sum_a Tr((t^{s_1}..t^{s_m})^dagger t^{s'_1}..t^{s'_m})
is computed here exactly by colour-flow loop counting: each adjoint pair is
replaced by the Fierz identity t^a_ij t^a_kl = (d_il d_kj - d_ij d_kl / N)/2,
and every resulting product of Kronecker deltas is N^(closed index loops).
"""
from __future__ import annotations

import functools
import itertools
import math
import os
import sys
from fractions import Fraction


# ------------------------------------------------------------------ colour
def _count_cycles(succ):
    seen = [False] * len(succ)
    n = 0
    for i in range(len(succ)):
        if not seen[i]:
            n += 1
            j = i
            while not seen[j]:
                seen[j] = True
                j = succ[j]
    return n


def trace_sum(word, N=3):
    """sum over repeated adjoint labels of Tr(t^{w_0} t^{w_1} ...), exact.

    Index slots: generator p has a row slot 2p and a column slot 2p+1; the
    trace joins column p to row p+1.  A Fierz term joins slots with deltas;
    the value of a delta network is N^(number of closed loops).
    """
    n = len(word)
    pairs = {}
    for p, a in enumerate(word):
        pairs.setdefault(a, []).append(p)
    plist = [tuple(v) for v in pairs.values()]
    assert all(len(v) == 2 for v in plist)
    total = Fraction(0)
    for choice in itertools.product((0, 1), repeat=len(plist)):
        # link[x] = the slot connected to x by a delta from a Fierz term
        link = [None] * (2 * n)
        coef = Fraction(1)
        for (p, q), c in zip(plist, choice):
            coef *= Fraction(1, 2)
            if c == 0:   # exchange term: row p - col q, row q - col p
                link[2 * p], link[2 * q + 1] = 2 * q + 1, 2 * p
                link[2 * q], link[2 * p + 1] = 2 * p + 1, 2 * q
            else:        # singlet term: row p - col p, row q - col q, times -1/N
                coef *= Fraction(-1, N)
                link[2 * p], link[2 * p + 1] = 2 * p + 1, 2 * p
                link[2 * q], link[2 * q + 1] = 2 * q + 1, 2 * q
        # follow loops: from a row slot go through its Fierz link to a column
        # slot, then along the trace to the next generator's row slot.
        succ = [0] * n
        for p in range(n):
            col = link[2 * p]
            succ[p] = (col // 2 + 1) % n
        total += coef * Fraction(N) ** _count_cycles(succ)
    return total


def multi_trace_sum(words, N=3):
    """sum over repeated adjoint labels of the product of traces
    Tr(t^{w_0} ...) Tr(t^{v_0} ...) ..., exact (every label appears twice;
    an empty word is a trace of the identity).  The same slot network as
    trace_sum, with the trace joins taken within each word."""
    pos = []  # (word index, position) of each generator, in order
    for wi, w_ in enumerate(words):
        for p_ in range(len(w_)):
            pos.append((wi, p_))
    n = len(pos)
    start = {}
    k = 0
    for wi, w_ in enumerate(words):
        start[wi] = k
        k += len(w_)
    labels = [w_[p_] for wi, w_ in enumerate(words) for p_ in range(len(w_))]
    pairs = {}
    for g, a in enumerate(labels):
        pairs.setdefault(a, []).append(g)
    plist = [tuple(v) for v in pairs.values()]
    assert all(len(v) == 2 for v in plist)
    empty = sum(1 for w_ in words if len(w_) == 0)
    total = Fraction(0)
    for choice in itertools.product((0, 1), repeat=len(plist)):
        link = [None] * (2 * n)
        coef = Fraction(1)
        for (p_, q_), c in zip(plist, choice):
            coef *= Fraction(1, 2)
            if c == 0:
                link[2 * p_], link[2 * q_ + 1] = 2 * q_ + 1, 2 * p_
                link[2 * q_], link[2 * p_ + 1] = 2 * p_ + 1, 2 * q_
            else:
                coef *= Fraction(-1, N)
                link[2 * p_], link[2 * p_ + 1] = 2 * p_ + 1, 2 * p_
                link[2 * q_], link[2 * q_ + 1] = 2 * q_ + 1, 2 * q_
        succ = [0] * n
        for g in range(n):
            col = link[2 * g] // 2
            wi, p_ = pos[col]
            succ[g] = start[wi] + (p_ + 1) % len(words[wi])
        total += coef * Fraction(N) ** (_count_cycles(succ) + empty)
    return total


# Colour tensors of the five diagrams of q q~ -> t t~ g (and, with the light
# line read from the outgoing quark, of q g -> t t~ q): a light-quark line L
# and the top line T joined by one gluon, and one external gluon of adjoint
# index "a".  Each is a sum of terms (coefficient, closed traces, L word,
# T word); f^{abc} = -2i Tr([t^a, t^b] t^c).
TWO_LINE_TENSORS = [
    [((1, 0), (), ("b", "a"), ("b",))],
    [((1, 0), (), ("a", "b"), ("b",))],
    [((1, 0), (), ("c",), ("a", "c"))],
    [((1, 0), (), ("c",), ("c", "a"))],
    [((0, -2), (("a", "b", "c"),), ("b",), ("c",)), ((0, 2), (("b", "a", "c"),), ("b",), ("c",))],
]


@functools.lru_cache(maxsize=None)
def two_line_colour_matrix():
    """CC[d][d'] = sum over all colours of C_d C_d'^* for the tensors above,
    as exact complex rationals (re, im): the conjugate of a string of
    generators is the reversed string, so every product closes into traces
    (L with L'^dagger, T with T'^dagger, each closed trace of C_d' reversed);
    the internal labels of d' are renamed, the external gluon's is shared."""
    def ren(w_):
        return tuple(x if x == "a" else x + "'" for x in w_)

    def cmul(a, b):
        return (a[0] * b[0] - a[1] * b[1], a[0] * b[1] + a[1] * b[0])

    out = []
    for d in TWO_LINE_TENSORS:
        row = []
        for e in TWO_LINE_TENSORS:
            re_, im_ = Fraction(0), Fraction(0)
            for c1, cl1, L1, T1 in d:
                for c2, cl2, L2, T2 in e:
                    coef = cmul((Fraction(c1[0]), Fraction(c1[1])), (Fraction(c2[0]), -Fraction(c2[1])))
                    words = list(cl1) + [tuple(reversed(ren(w_))) for w_ in cl2]
                    words.append(tuple(L1) + tuple(reversed(ren(L2))))
                    words.append(tuple(T1) + tuple(reversed(ren(T2))))
                    v = multi_trace_sum(words)
                    re_ += coef[0] * v
                    im_ += coef[1] * v
            row.append((re_, im_))
        out.append(row)
    return out


@functools.lru_cache(maxsize=None)
def colour_matrix(m):
    perms = list(itertools.permutations(range(m)))
    C = [[trace_sum(tuple(reversed(s)) + sp) for sp in perms] for s in perms]
    den = 1
    for row in C:
        for v in row:
            den = den * v.denominator // math.gcd(den, v.denominator)
    Z = [[int(v * den) for v in row] for row in C]
    return perms, Z, den


# ---------------------------------------------------------------- emitter
def _name(seq):
    return "".join(str(i) for i in seq)


def _mask(seq):
    return sum(1 << i for i in seq)


def _vsum(t3, t4):
    """Sum of three-gluon vertices minus four-gluon vertices as one nested
    accumulation (v3, then v3_acc for the other v3 terms, then w4_sub): every
    component is a single chain of fused multiply-adds.  t3: tuples
    (X, Y, PX, PY); t4: tuples (A, B, C)."""
    e = f"v3({', '.join(t3[0])})"
    for a in t3[1:]:
        e = f"v3_acc({', '.join(a)}, {e})"
    for a in t4:
        e = f"w4_sub({', '.join(a)}, {e})"
    return e


def _ssum(terms):
    """Sum of slashed currents on spinors, (J, S) tuples, as one accumulation."""
    e = f"slash({terms[0][0]}, {terms[0][1]})"
    for J_, S_ in terms[1:]:
        e = f"slash_acc({J_}, {S_}, {e})"
    return e


def _colour_lines(w, ind, groups, name):
    """total += sum over coefficient groups c * (sum of |A_i|^2 or
    Re(A_i^* A_j)); each group's sum is one chain of fused multiply-adds.
    name(i) is the amplitude variable of ordering i."""
    for c, lst in sorted(groups.items()):
        calls = []
        for k_, (i, j) in enumerate(lst):
            if k_ == 0:
                first = f"cabs2({name(i)})" if i == j else f"cre_dot({name(i)}, {name(j)})"
                continue
            calls.append(f"s = cabs2_acc({name(i)}, s);" if i == j else f"s = cre_dot_acc({name(i)}, {name(j)}, s);")
        w(f"{ind}{{")
        w(f"{ind}  R s = {first};")
        for q in range(0, len(calls), 3):
            w(f"{ind}  " + " ".join(calls[q:q + 3]))
        w(f"{ind}  total = total + R({c}.0) * s;")
        w(f"{ind}}}")


# Real-flop cost of each device routine in amp.h (a fused multiply-add counts
# as two flops): Minkowski product 7; v3 47 (three Minkowski products, the
# conserved currents' PX.X and PY.Y being zero); w4 42; scaling a four-vector 4;
# adding four-vectors 4; slash(real J, spinor) 42; prop 63 (five coefficient
# products, two sums, then 8 x (one product + three fused multiply-adds));
# adding spinors 8; ubar_dot 30; cabs2 and cre_dot 3.  The accumulating forms
# (v3_acc, w4_sub, slash_acc, cabs2_acc, cre_dot_acc) cost exactly the plain
# routine plus the addition they absorb.
COST = {"v3": 47, "w4": 42, "vscale": 4, "vadd": 4, "slash": 42, "prop": 63, "sadd": 8, "ubar": 30,
        "abs2": 3, "redot": 3, "mdot": 7}


def flop_count(m: int) -> dict:
    """Static flop count per event of the generated |M|^2 with the currents
    shared across colour orderings (per-event constants, then for every
    antitop helicity and gluon polarisation state the currents, partial
    amplitudes and colour form; where the schedule shares the gluon currents
    between the two antitop helicities they are counted once per gluon
    polarisation state)."""
    return emit_me(m, with_cost=True)[1]


def emit_me(m: int, with_cost: bool = False):
    cost = {"const": 0, "body": 0, "gluon": 0}
    perms, Z, den = colour_matrix(m)
    nf = len(perms)
    L = []
    w = L.append
    w(f"// Generated by gen_me.py for g g -> t t~ + {m - 2} g ({m} gluons on the top line,")
    w(f"// {nf} colour orderings, {1 << (m + 2)} helicity/polarisation states). Do not edit.")
    w("#pragma once")
    w('#include "amp.h"')
    w("namespace mf {")
    w(f"constexpr int ME_M{m}_NF = {nf};")
    w(f"constexpr double ME_M{m}_COLOUR_DEN = {den}.0;")
    w("// Colour- and polarisation-summed |M|^2 with g = 1.")
    w("//   K[i]: outgoing gluon momenta (i = 0,1 the crossed beams), E[i][l]: the two")
    w("//   real polarisation vectors of gluon i; UB[l]: ubar(top) for the two top")
    w("//   helicities; VS[l]: v(antitop); PTB: antitop momentum; MT: top mass.")
    w("//   Per-event invariants and propagator factors are formed in the kinematic")
    w("//   type RK (FP64) and only then converted to the amplitude type R, so that")
    w("//   denominators such as (p_t + k)^2 - m^2 = 2 p_t.k + k^2 never cancel in R.")
    w("template <class R, class RK>")
    w(f"__device__ __forceinline__ R me_gg_m{m}(const V4<RK>* K, const V4<R> (*E)[2], const Sp<R>* UB,")
    w("                                         const Sp<R>* VS, const V4<RK>& PTB, RK MTK) {")
    w("  const R MT = cvt<R>(MTK);")
    subsets = [s for s in range(1, 1 << m)]
    for s_ in subsets:
        idx = [i for i in range(m) if s_ >> i & 1]
        if len(idx) == 1:
            w(f"  const V4<RK> PK{s_} = K[{idx[0]}];")
        else:
            w(f"  const V4<RK> PK{s_} = " + " + ".join(f"K[{i}]" for i in idx) + ";")
        w(f"  const V4<R> P{s_} = cvt4<R>(PK{s_});")
    for s_ in subsets:
        if bin(s_).count("1") >= 2:
            w(f"  const R G{s_} = cvt<R>(RK(-1.0) / mdot(PK{s_}, PK{s_}));")
            cost["const"] += COST["vadd"] * (bin(s_).count("1") - 1) + COST["mdot"] + 1
    full = (1 << m) - 1
    for s_ in subsets:
        if s_ != full:
            w(f"  const V4<R> Q{s_} = cvt4<R>(RK(-1.0) * (PTB + PK{s_}));")
            w(f"  const R IQ{s_} = cvt<R>(RK(-1.0) / (RK(2.0) * mdot(PTB, PK{s_}) + mdot(PK{s_}, PK{s_})));")
            cost["const"] += 2 * COST["vadd"] + 2 * COST["mdot"] + 3
    w("  R total = R(0.0);")
    # antitop helicity outermost: nothing but the per-event constants above is
    # invariant across the inner loop, which keeps every current's live range
    # inside one polarisation state.
    w("#pragma unroll 1")
    w("  for (int ht = 0; ht < 2; ++ht) {")
    w("    const Sp<R> S_ = VS[ht];")
    w("#pragma unroll 1")
    w(f"    for (int hg = 0; hg < {1 << m}; ++hg) {{")
    ind = "      "
    for i in range(m):
        w(f"{ind}const V4<R> J{i} = ((hg >> {m - 1 - i}) & 1) ? E[{i}][1] : E[{i}][0];")
    emitted = set(f"J{i}" for i in range(m)) | {"S_"}

    def need_J(seq):
        nm = f"J{_name(seq)}"
        if nm in emitted:
            return nm
        rev = f"J{_name(seq[::-1])}"
        if rev in emitted:
            # reflection of a colour-ordered current: J(n..1) = (-1)^(n+1) J(1..n),
            # no arithmetic (a sign flip folds into the consumers)
            if len(seq) % 2 == 1:
                return rev
            w(f"{ind}const V4<R> {nm} = R(-1.0) * {rev};")
            emitted.add(nm)
            return nm
        terms3 = []
        for j in range(1, len(seq)):
            a, b = seq[:j], seq[j:]
            terms3.append((need_J(a), need_J(b), f"P{_mask(a)}", f"P{_mask(b)}"))
        terms4 = []
        for j in range(1, len(seq) - 1):
            for l in range(j + 1, len(seq)):
                a, b, c = seq[:j], seq[j:l], seq[l:]
                terms4.append((need_J(a), need_J(b), need_J(c)))
        w(f"{ind}const V4<R> {nm} = G{_mask(seq)} * ({_vsum(terms3, terms4)});")
        c_ = (len(terms3) * COST["v3"] + len(terms4) * COST["w4"]
              + (len(terms3) + len(terms4) - 1) * COST["vadd"] + COST["vscale"])
        cost["body"] += c_
        cost["gluon"] += c_
        emitted.add(nm)
        return nm

    def need_S(seq):
        nm = f"S_{_name(seq)}"
        if nm in emitted:
            return nm
        terms = []
        for j in range(1, len(seq) + 1):
            a, b = seq[:j], seq[j:]
            terms.append((need_J(a), need_S(b)))
        s_ = _mask(seq)
        w(f"{ind}const Sp<R> {nm} = prop(Q{s_}, MT, IQ{s_}, {_ssum(terms)});")
        cost["body"] += len(terms) * COST["slash"] + (len(terms) - 1) * COST["sadd"] + COST["prop"]
        emitted.add(nm)
        return nm

    for k, seq in enumerate(perms):
        terms = []
        for j in range(1, m + 1):
            a, b = seq[:j], seq[j:]
            terms.append((need_J(a), need_S(b)))
        w(f"{ind}const Sp<R> F{k} = {_ssum(terms)};")
        cost["body"] += len(terms) * COST["slash"] + (len(terms) - 1) * COST["sadd"]
        for t in range(2):
            w(f"{ind}const C2<R> A{t}_{k} = ubar_dot(UB[{t}], F{k});")
            cost["body"] += COST["ubar"]
    groups = {}
    for i in range(nf):
        for j in range(i, nf):
            c = Z[i][j] * (1 if i == j else 2)
            groups.setdefault(c, []).append((i, j))
    for t in range(2):
        _colour_lines(w, ind, groups, lambda i, t=t: f"A{t}_{i}")
        for c, lst in sorted(groups.items()):
            cost["body"] += 3 * len(lst) + (len(lst) - 1) + 2
    w("    }")
    w("  }")
    w(f"  return total * R(1.0 / {den}.0);")
    w("}")
    w("}  // namespace mf")
    text = "\n".join(L) + "\n"
    if with_cost:
        n_states = 2 * (1 << m)
        out = {"per_event_constants": cost["const"], "per_state": cost["body"], "states": n_states,
               "total": cost["const"] + n_states * cost["body"]}
        if SCHEDULE.get(m) == "per_ordering_shared_antitop":
            # the gluon currents do not depend on the antitop helicity and are
            # built once per gluon polarisation state
            out["gluon_currents_per_polarisation"] = cost["gluon"]
            out["total"] -= (n_states // 2) * cost["gluon"]
        return text, out
    return text


def emit_me_per_ordering(m: int, share_antitop: bool = False, pair_orderings=False, suffix: str = "") -> str:
    """Lower-register schedule: each colour ordering builds its own currents.

    Only per-event scalars (propagator factors, formed in the kinematic type),
    spinors, polarisation vectors and momenta live across the loops.  Inside a
    polarisation state every ordering starts from fresh opaque copies of the
    external currents and momenta, so the compiler cannot merge currents across
    orderings and each ordering's intermediates die before the next begins.
    The amplitudes A[ordering][top helicity] stay in registers for the colour
    form.  Extra work versus sharing currents across orderings: the
    sub-sequence currents and antitop currents are rebuilt per ordering.
    share_antitop: the gluon currents of an ordering are built once per gluon
    polarisation state and used for both antitop helicities (the antitop
    spinor enters only the top-line currents), at the cost of holding the
    amplitudes of both antitop helicities until the colour form.
    """
    perms, Z, den = colour_matrix(m)
    nf = len(perms)
    L = []
    w = L.append
    w(f"// Generated by gen_me.py for g g -> t t~ + {m - 2} g ({m} gluons on the top line,")
    w(f"// {nf} colour orderings, {1 << (m + 2)} helicity/polarisation states),")
    grouping = {"all": "all orderings in one block", "last": "orderings grouped by their last gluon",
                True: "orderings in pairs"}.get(pair_orderings, "one ordering at a time")
    w(f"// per-ordering schedule, {grouping}. Do not edit.")
    w("#pragma once")
    w('#include "amp.h"')
    w("namespace mf {")
    if not suffix:
        w(f"constexpr int ME_M{m}_NF = {nf};")
        w(f"constexpr double ME_M{m}_COLOUR_DEN = {den}.0;")
    w("// Colour- and polarisation-summed |M|^2 with g = 1 (argument meaning as in")
    w("// the shared-current schedule).")
    w("template <class R, class RK>")
    w(f"__device__ __forceinline__ R me_gg_m{m}{suffix}(const V4<RK>* K, const V4<R> (*E)[2], const Sp<R>* UB,")
    w("                                         const Sp<R>* VS, const V4<RK>& PTB, RK MTK) {")
    w("  const R MT = cvt<R>(MTK);")
    subsets = list(range(1, 1 << m))
    full = (1 << m) - 1

    def ksum(s_, pref="K"):
        idx = [i for i in range(m) if s_ >> i & 1]
        return " + ".join(f"{pref}[{i}]" if pref == "K" else f"{pref}{i}" for i in idx)

    for s_ in subsets:
        if bin(s_).count("1") >= 2:
            w(f"  R G{s_};")
            w(f"  {{ const V4<RK> P = {ksum(s_)}; G{s_} = cvt<R>(RK(-1.0) / mdot(P, P)); }}")
    for s_ in subsets:
        if s_ != full:
            w(f"  R IQ{s_};")
            w(f"  {{ const V4<RK> P = {ksum(s_)}; IQ{s_} = cvt<R>(RK(-1.0) / (RK(2.0) * mdot(PTB, P) + mdot(P, P))); }}")
    for i in range(m):
        w(f"  const V4<R> K{i} = cvt4<R>(K[{i}]);")
    w("  const V4<R> PB = cvt4<R>(PTB);")
    w("  R total = R(0.0);")
    hts = (0, 1) if share_antitop else (None,)
    if not share_antitop:
        w("#pragma unroll 1")
        w("  for (int ht = 0; ht < 2; ++ht) {")
        w("    const Sp<R> V = VS[ht];")
    else:
        w("  {")
    w("#pragma unroll 1")
    w(f"    for (int hg = 0; hg < {1 << m}; ++hg) {{")
    ind = "      "
    for i in range(m):
        w(f"{ind}const V4<R> E{i} = ((hg >> {m - 1 - i}) & 1) ? E[{i}][1] : E[{i}][0];")
    # orderings handled together: pairs that differ by the swap of their
    # first two gluons share the currents of positions 2.. (gluon and top-line
    # spinor currents), and their leading two-gluon currents differ in sign
    # each block is a list of sub-blocks: the gluon currents of a sub-block
    # are built, then its top-line currents for each antitop helicity, before
    # the next sub-block starts; whatever the sub-blocks of one block share is
    # built once
    index = {seq: k for k, seq in enumerate(perms)}
    pairs = [(k, index[(seq[1], seq[0]) + seq[2:]]) for k, seq in enumerate(perms)]
    pairs = [pr for pr in pairs if pr[0] < pr[1]]
    if pair_orderings == "all":
        order = [[tuple(range(nf))]]
    elif pair_orderings == "last":
        order = [[pr for pr in pairs if perms[pr[0]][-1] == d] for d in range(m)]
    elif pair_orderings:
        order = [[pr] for pr in pairs]
    else:
        order = [[(k,)] for k in range(nf)]
    for block in order:
        grp = [k for sub in block for k in sub]
        for k in grp:
            for h in hts:
                hs = "" if h is None else f"h{h}"
                w(f"{ind}C2<R> A0{hs}_{k}, A1{hs}_{k};")
        w(f"{ind}{{  // ordering" + ("s " if len(grp) > 1 else " ") + ", ".join(str(perms[k]) for k in grp))
        ii = ind + "  "
        for i in range(m):
            w(f"{ii}V4<R> J{i} = E{i}; opaque4(J{i});")
            w(f"{ii}V4<R> k{i} = K{i}; opaque4(k{i});")
        if not share_antitop:
            w(f"{ii}Sp<R> S_ = V; opaque_sp(S_);")
        w(f"{ii}V4<R> pb = PB; opaque4(pb);")
        done = set(f"J{i}" for i in range(m)) | ({"S_"} if not share_antitop else set())
        psum = set()

        def P(sq):
            s_ = _mask(sq)
            nm = f"p{s_}"
            if len(sq) == 1:
                return f"k{sq[0]}"
            if nm not in psum:
                w(f"{ii}const V4<R> {nm} = " + " + ".join(f"k{i}" for i in sorted(sq)) + ";")
                psum.add(nm)
            return nm

        def J(sq):
            nm = f"J{_name(sq)}"
            if nm in done:
                return nm
            rev = f"J{_name(sq[::-1])}"
            if rev in done:
                # reflection of a colour-ordered current: J(n..1) = (-1)^(n+1) J(1..n)
                if len(sq) % 2 == 0:
                    w(f"{ii}const V4<R> {nm} = R(-1.0) * {rev};")
                    done.add(nm)
                    return nm
                return rev
            t3 = [(J(sq[:j]), J(sq[j:]), P(sq[:j]), P(sq[j:])) for j in range(1, len(sq))]
            t4 = [(J(sq[:j]), J(sq[j:l]), J(sq[l:])) for j in range(1, len(sq) - 1)
                  for l in range(j + 1, len(sq))]
            w(f"{ii}const V4<R> {nm} = G{_mask(sq)} * ({_vsum(t3, t4)});")
            done.add(nm)
            return nm

        def S(sq, hs):
            nm = f"S{hs}_{_name(sq)}"
            if nm in done:
                return nm
            terms = [(J(sq[:j]), S(sq[j:], hs)) for j in range(1, len(sq) + 1)]
            s_ = _mask(sq)
            w(f"{ii}const Sp<R> {nm} = prop_neg(pb + {P(sq)}, MT, IQ{s_}, {_ssum(terms)});")
            done.add(nm)
            return nm

        # with share_antitop: the gluon currents first (shared by both antitop
        # helicities), then the top line for each antitop helicity
        for sub in block:
            if share_antitop:
                for k in sub:
                    for j in range(1, m + 1):
                        J(perms[k][:j])
            for h in hts:
                hs = "" if h is None else f"h{h}"
                if share_antitop and f"S{hs}_" not in done:
                    w(f"{ii}Sp<R> S{hs}_ = VS[{h}]; opaque_sp(S{hs}_);")
                    done.add(f"S{hs}_")
                for k in sub:
                    seq = perms[k]
                    terms = [(J(seq[:j]), S(seq[j:], hs)) for j in range(1, m + 1)]
                    w(f"{ii}const Sp<R> F{hs}_{k} = {_ssum(terms)};")
                    w(f"{ii}A0{hs}_{k} = ubar_dot(UB[0], F{hs}_{k});")
                    w(f"{ii}A1{hs}_{k} = ubar_dot(UB[1], F{hs}_{k});")
        w(f"{ind}}}")
    groups = {}
    for i in range(nf):
        for j in range(i, nf):
            c = Z[i][j] * (1 if i == j else 2)
            groups.setdefault(c, []).append((i, j))
    for h in hts:
        hs = "" if h is None else f"h{h}"
        for t in range(2):
            _colour_lines(w, ind, groups, lambda i, t=t, hs=hs: f"A{t}{hs}_{i}")
    w("    }")
    w("  }")
    w(f"  return total * R(1.0 / {den}.0);")
    w("}")
    w("}  // namespace mf")
    return "\n".join(L) + "\n"


def emit_amp_store(m: int) -> str:
    """Partial amplitudes of m gluons for a range of gluon polarisation
    states, stored for a separate colour sum (no colour form here): the same
    per-ordering Berends-Giele steps, and the same sharing of each ordering's
    gluon currents between the two antitop helicities, as
    emit_me_per_ordering(m, share_antitop=True).  The per-event constants
    (propagator factors, polarisation vectors, momenta, antitop spinors) are
    read from per-lane LDS tables inside each ordering, through an opaque
    zero offset, so that they do not stay live in registers across the
    orderings.  For gluon state hg, antitop helicity h and top helicity t the
    amplitude of ordering k goes to
      out[slice * sstride + (k / 4) * ld4 + k % 4],
      slice = (((hg - hg0) * 2 + h) * 2 + t) * 2 + (0: re, 1: im).
    Tables (each pointer already at the lane's column, stride AW):
      gt[S * AW]: -1 / P_S^2 for gluon subsets S with >= 2 gluons;
      qt[S * AW]: -1 / ((p_tb + P_S)^2 - m_t^2) for S != all;
      et[(2 i + p) * AW]: polarisation p of gluon i; kt[i * AW]: momentum of
      gluon i; vt[h * AW]: v(antitop) of helicity h."""
    perms, Z, den = colour_matrix(m)
    nf = len(perms)
    L = []
    w = L.append
    w(f"// Generated by gen_me.py for g g -> t t~ + {m - 2} g ({m} gluons on the top line,")
    w(f"// {nf} colour orderings, {4 << m} helicity/polarisation states): partial")
    w("// amplitudes stored for the colour sum on the matrix cores. Do not edit.")
    w("#pragma once")
    w('#include "amp.h"')
    w("namespace mf {")
    w(f"constexpr int AMPS_M{m}_NF = {nf};")
    w(f"constexpr int AMPS_M{m}_NQ = {nf // 4};  // groups of four orderings")
    w(f"constexpr int AMPS_M{m}_HG = {1 << m};  // gluon polarisation states")
    w("template <class R, int AW>")
    w(f"__device__ __forceinline__ void amp_gg_m{m}_store(const R* gt, const R* qt, const V4<R>* et, const V4<R>* kt,")
    w("                                               const Sp<R>* vt, const Sp<R>* UB, const V4<R>& PB, R MT,")
    w("                                               int hg0, int nhg, R* out, int64_t sstride, int64_t ld4) {")
    w("#pragma unroll 1")
    w("  for (int hg = hg0; hg < hg0 + nhg; ++hg) {")
    w("    R* const o_hg = out + (int64_t)((hg - hg0) * 8) * sstride;")
    ind = "    "
    for k, seq in enumerate(perms):
        w(f"{ind}{{  // ordering {seq}")
        ii = ind + "  "
        w(f"{ii}int z_ = 0;")
        w(f"{ii}asm volatile(\"\" : \"+v\"(z_));")
        for i in range(m):
            w(f"{ii}const V4<R> J{i} = et[(2 * {i} + ((hg >> {m - 1 - i}) & 1)) * AW + z_];")
            w(f"{ii}const V4<R> k{i} = kt[{i} * AW + z_];")
        w(f"{ii}V4<R> pb = PB;")
        w(f"{ii}opaque4(pb);")
        done = set(f"J{i}" for i in range(m))
        psum = set()
        consts = set()

        def P(sq):
            s_ = _mask(sq)
            nm = f"p{s_}"
            if len(sq) == 1:
                return f"k{sq[0]}"
            if nm not in psum:
                w(f"{ii}const V4<R> {nm} = " + " + ".join(f"k{i}" for i in sorted(sq)) + ";")
                psum.add(nm)
            return nm

        def G(sq):
            s_ = _mask(sq)
            if f"G{s_}" not in consts:
                w(f"{ii}const R G{s_} = gt[{s_} * AW + z_];")
                consts.add(f"G{s_}")
            return f"G{s_}"

        def IQ(sq):
            s_ = _mask(sq)
            if f"IQ{s_}" not in consts:
                w(f"{ii}const R IQ{s_} = qt[{s_} * AW + z_];")
                consts.add(f"IQ{s_}")
            return f"IQ{s_}"

        def J(sq):
            nm = f"J{_name(sq)}"
            if nm in done:
                return nm
            t3 = [(J(sq[:j]), J(sq[j:]), P(sq[:j]), P(sq[j:])) for j in range(1, len(sq))]
            t4 = [(J(sq[:j]), J(sq[j:l]), J(sq[l:])) for j in range(1, len(sq) - 1)
                  for l in range(j + 1, len(sq))]
            g = G(sq)
            w(f"{ii}const V4<R> {nm} = {g} * ({_vsum(t3, t4)});")
            done.add(nm)
            return nm

        def S(sq, hs):
            nm = f"S{hs}_{_name(sq)}"
            if nm in done:
                return nm
            terms = [(J(sq[:j]), S(sq[j:], hs)) for j in range(1, len(sq) + 1)]
            q = IQ(sq)
            w(f"{ii}const Sp<R> {nm} = prop_neg(pb + {P(sq)}, MT, {q}, {_ssum(terms)});")
            done.add(nm)
            return nm

        for j in range(1, m + 1):
            J(seq[:j])
        for h in (0, 1):
            hs = f"h{h}"
            w(f"{ii}const Sp<R> S{hs}_ = vt[{h} * AW + z_];")
            done.add(f"S{hs}_")
            terms = [(J(seq[:j]), S(seq[j:], hs)) for j in range(1, m + 1)]
            w(f"{ii}const Sp<R> F{hs} = {_ssum(terms)};")
            w(f"{ii}{{")
            w(f"{ii}  const C2<R> a0 = ubar_dot(UB[0], F{hs}), a1 = ubar_dot(UB[1], F{hs});")
            w(f"{ii}  R* o_ = o_hg + (int64_t)({h * 4}) * sstride + (int64_t)({k >> 2}) * ld4 + {k & 3};")
            w(f"{ii}  o_[0] = a0.re;")
            w(f"{ii}  o_[sstride] = a0.im;")
            w(f"{ii}  o_[2 * sstride] = a1.re;")
            w(f"{ii}  o_[3 * sstride] = a1.im;")
            w(f"{ii}}}")
        w(f"{ind}}}")
    w("  }")
    w("}")
    vals = ", ".join(str(v) for row in Z for v in row)
    w(f"// colour matrix numerators C[s][s'] * {den}, row-major")
    w(f"constexpr double AMPS_M{m}_COLOUR_DEN = {den}.0;")
    w(f"__device__ const float AMPS_M{m}_COLOUR[{nf * nf}] = {{{vals}}};")
    w("}  // namespace mf")
    return "\n".join(L) + "\n"


def emit_colour_qq() -> str:
    """The colour matrix of the five diagrams of the two-quark-line channels
    (q q~ -> t t~ g, q g -> t t~ q) over a common denominator."""
    CC = two_line_colour_matrix()
    den = 1
    for row in CC:
        for re_, im_ in row:
            for v in (re_, im_):
                den = den * v.denominator // math.gcd(den, v.denominator)
    re_s = ", ".join(f"{int(re_ * den)}.0" for row in CC for re_, _ in row)
    im_s = ", ".join(f"{int(im_ * den)}.0" for row in CC for _, im_ in row)
    L = ["// Generated by gen_me.py: colour matrix CC[d][d'] = sum_colours C_d C_d'^* of the",
         "// five diagrams of q q~ -> t t~ g and q g -> t t~ q (two quark lines joined by a",
         "// gluon, one more external gluon), by colour-flow loop counting.  Do not edit.",
         "#pragma once",
         "namespace mf {",
         f"constexpr double QQ_CC_DEN = {den}.0;",
         f"__device__ const double QQ_CC_RE[25] = {{{re_s}}};",
         f"__device__ const double QQ_CC_IM[25] = {{{im_s}}};",
         "}  // namespace mf"]
    return "\n".join(L) + "\n"


def emit_amp_tables(m: int) -> str:
    """Tables for the streamed partial amplitudes of m gluons (the per-ordering
    routine itself is hand-written in gg3.h):

    * AMP_M{m}_SIGMA[k][i]: gluon at position i of colour ordering k
      (orderings in lexicographic order, as the colour matrix);
    * AMP_M{m}_GMASK[k][r]: gluon subset of the r-th contiguous range of
      positions (ranges of length >= 2 in the order (0,1), (1,2), ..., by
      length then start), whose propagator factor the range's current uses;
    * AMP_M{m}_QMASK[k][j]: gluon subset of the suffix starting at position
      j + 1, whose top propagator closes the suffix's spinor current;
    * AMP_M{m}_COLOUR: colour matrix numerators C[s][s'] * den, row-major.
    """
    perms, Z, den = colour_matrix(m)
    nf = len(perms)
    nfp = (nf + 15) // 16 * 16
    ranges = [(a, a + ln - 1) for ln in range(2, m + 1) for a in range(0, m - ln + 1)]
    L = []
    w = L.append
    w(f"// Generated by gen_me.py for g g -> t t~ + {m - 2} g ({m} gluons on the top line,")
    w(f"// {nf} colour orderings, {2 << m} helicity/polarisation states): tables of the")
    w("// streamed partial amplitudes. Do not edit.")
    w("#pragma once")
    w("#include <stdint.h>")
    w("namespace mf {")
    w(f"constexpr int AMP_M{m}_NF = {nf};")
    w(f"constexpr int AMP_M{m}_NQ = {nfp // 4};  // four-ordering groups incl. zero padding")
    w(f"constexpr int AMP_M{m}_STATES = {2 << m};")
    w(f"constexpr int AMP_M{m}_NRANGE = {len(ranges)};")
    w(f"constexpr double AMP_M{m}_COLOUR_DEN = {den}.0;")
    w("// contiguous ranges (first, last position) in table order")
    w(f"constexpr int AMP_M{m}_RANGE[{len(ranges)}][2] = {{" + ", ".join(f"{{{a}, {b}}}" for a, b in ranges) + "};")
    sig = ", ".join("{" + ", ".join(str(i) for i in p_) + "}" for p_ in perms)
    w(f"__device__ const uint8_t AMP_M{m}_SIGMA[{nf}][{m}] = {{{sig}}};")
    gm = ", ".join("{" + ", ".join(str(sum(1 << p_[i] for i in range(a, b + 1))) for a, b in ranges) + "}"
                   for p_ in perms)
    w(f"__device__ const uint8_t AMP_M{m}_GMASK[{nf}][{len(ranges)}] = {{{gm}}};")
    qm = ", ".join("{" + ", ".join(str(sum(1 << p_[i] for i in range(j, m))) for j in range(1, m)) + "}"
                   for p_ in perms)
    w(f"__device__ const uint8_t AMP_M{m}_QMASK[{nf}][{m - 1}] = {{{qm}}};")
    # orderings that differ by the swap of their first two gluons share every
    # current of the last m - 2 positions: pairs (a, b), a < b
    index = {p_: k for k, p_ in enumerate(perms)}
    pairs = []
    for k, p_ in enumerate(perms):
        q_ = (p_[1], p_[0]) + tuple(p_[2:])
        if k < index[q_]:
            pairs.append((k, index[q_]))
    w(f"constexpr int AMP_M{m}_NPAIR = {len(pairs)};")
    w(f"__device__ const uint8_t AMP_M{m}_PAIR[{len(pairs)}][2] = {{" + ", ".join(f"{{{a}, {b}}}" for a, b in pairs)
      + "};")
    vals = ", ".join(str(v) for row in Z for v in row)
    w(f"__device__ const float AMP_M{m}_COLOUR[{nf * nf}] = {{{vals}}};")
    w("}  // namespace mf")
    return "\n".join(L) + "\n"


def amp_flop_count(m: int) -> dict:
    """Static flop count per event of the streamed partial amplitudes plus the
    colour sum over the unpadded orderings (the algorithm as emitted: per
    ordering, less what each pair of orderings shares).  A single state
    costs amplitudes_single_state; the sum over all states builds the gluon
    currents of each gluon polarisation state once for both antitop
    helicities, so its average per state is amplitudes_per_state."""
    perms, _, _ = colour_matrix(m)
    body = 0
    gluon = 0
    for seq in perms:
        done = set()

        def J(sq):
            nonlocal body, gluon
            if len(sq) == 1 or sq in done:
                return
            n3 = len(sq) - 1
            n4 = (len(sq) - 1) * (len(sq) - 2) // 2
            for j in range(1, len(sq)):
                J(sq[:j])
                J(sq[j:])
            c_ = n3 * COST["v3"] + n4 * COST["w4"] + (n3 + n4 - 1) * COST["vadd"] + COST["vscale"]
            body += c_
            gluon += c_
            done.add(sq)

        def S(sq):
            nonlocal body
            if not sq or sq in done:
                return
            for j in range(1, len(sq) + 1):
                J(sq[:j])
                S(sq[j:])
            body += len(sq) * COST["slash"] + (len(sq) - 1) * COST["sadd"] + COST["prop"]
            done.add(sq)

        for j in range(1, m + 1):
            J(seq[:j])
            S(seq[j:])
        body += m * COST["slash"] + (m - 1) * COST["sadd"] + 2 * COST["ubar"]
    # pairs of orderings that differ by the swap of the first two gluons
    # compute the currents of positions 2..m-1 once: the gluon currents of
    # the ranges inside them and the spinor currents of the suffixes from 2
    shared = 0
    for ln in range(2, m - 1):
        n3, n4 = ln - 1, (ln - 1) * (ln - 2) // 2
        shared += (m - 2 - ln + 1) * (n3 * COST["v3"] + n4 * COST["w4"] + (n3 + n4 - 1) * COST["vadd"]
                                      + COST["vscale"])
    gluon_shared = shared
    for ln in range(1, m - 1):
        shared += ln * COST["slash"] + (ln - 1) * COST["sadd"] + COST["prop"]
    body -= (len(perms) // 2) * shared
    gluon -= (len(perms) // 2) * gluon_shared
    nf = len(perms)
    colour = 2 * 2 * (2 * nf * nf)  # two top helicities, real and imaginary parts, C times A and the dot
    states = 2 << m
    per_state = body - gluon // 2
    return {"amplitudes_per_state": per_state, "amplitudes_single_state": body,
            "gluon_currents_per_state": gluon, "colour_per_state": colour, "states": states,
            "total": states * (per_state + colour)}


SCHEDULE = {2: "memo", 3: "per_ordering_shared_antitop", 4: "per_ordering_shared_antitop", 5: "amplitudes"}
# per-ordering schedules that handle the orderings in pairs sharing their
# suffix currents ("all": every ordering in one block, so that besides the
# suffix currents the reflected currents J(n..1) = (-1)^(n+1) J(1..n) are
# shared too)
PAIR_ORDERINGS = {2: False, 3: "all", 4: True, 5: False}
# a second function with a wider grouping, me_gg_m4_grouped (the six orderings
# that end with the same gluon in one block), for the FP32 amplitudes: it needs
# more registers, which the FP32 kernel has and the FP64 one does not


def main(outdir: str, ms=(2, 3, 4, 5)) -> None:
    os.makedirs(outdir, exist_ok=True)
    for m in ms:
        if SCHEDULE[m] == "amplitudes":
            path = os.path.join(outdir, f"amp_gg_m{m}.h")
            text = emit_amp_tables(m)
        else:
            path = os.path.join(outdir, f"me_gg_m{m}.h")
            text = emit_me(m) if SCHEDULE[m] == "memo" else emit_me_per_ordering(
                m, share_antitop=SCHEDULE[m] == "per_ordering_shared_antitop", pair_orderings=PAIR_ORDERINGS[m])
        old = open(path).read() if os.path.exists(path) else None
        if old != text:
            with open(path, "w") as f:
                f.write(text)
    # g g -> t t~ g g: the wider grouping for FP32; the amplitudes stored for
    # the matrix-core colour sum; the colour matrix of the quark channels
    for name, text in (("me_gg_m4_grouped.h", emit_me_per_ordering(4, True, "last", "_grouped")),
                       ("amps_gg_m4.h", emit_amp_store(4)), ("colour_qq.h", emit_colour_qq())):
        path = os.path.join(outdir, name)
        old = open(path).read() if os.path.exists(path) else None
        if old != text:
            with open(path, "w") as f:
                f.write(text)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else os.path.join(os.path.dirname(__file__), "..", "csrc", "gen"))
