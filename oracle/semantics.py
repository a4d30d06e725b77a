"""ORACLE -- test infrastructure, not part of the product.

Dense brute-force statement of the GraphBLAS operations the paper uses
(Section III: Table I operations, Table II semirings, "Masks and
accumulators", "Masks"), for tiny inputs, in pure Python loops.

Objects are dictionaries of present entries: a matrix is
``Mat(nrows, ncols, {(i, j): value}, kind)`` and a vector is
``Vec(n, {i: value}, kind)``; kind is "bool" (pattern only, every value
1), "int32", "int64" or "fp64".  The paper leaves the domains to the
GraphBLAS C API, where an int32 result is taken modulo 2^32: each stage
here (a product's entries, a write's stored values, a reduction) takes its
int32 results modulo 2^32 into [-2^31, 2^31).

The `any` monoid may return any one of the candidates (Section IV-A), so a
result entry produced by it is an ``AnyOf`` holding every admissible value
unless ``deterministic`` asks for the smallest.

Readings taken where the paper is silent (it defers the mask/accumulator
interplay to the GraphBLAS specification):
  * T(i,j) exists iff at least one k has A'(i,k) and B'(k,j); the additive
    identity is never stored (the identity of min is +inf, Table II prints
    -inf).
  * Z = T without an accumulator, else the union of C and T with
    accum(C, T) where both exist.
  * Where the mask is true, C(i,j) = Z(i,j) if present and is deleted
    otherwise; where it is false, C(i,j) keeps its old value, or is deleted
    under replace.  A complemented empty mask is false everywhere.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field


class AnyOf:
    """A value known only up to membership in a candidate set."""

    __slots__ = ("c",)

    def __init__(self, cands):
        self.c = frozenset(cands)

    def __repr__(self):
        return f"AnyOf({sorted(self.c)})"


def _lift(op, x, y):
    xs = x.c if isinstance(x, AnyOf) else (x,)
    ys = y.c if isinstance(y, AnyOf) else (y,)
    res = {op(a, b) for a in xs for b in ys}
    return AnyOf(res) if len(res) > 1 else next(iter(res))


@dataclass
class Mat:
    nrows: int
    ncols: int
    e: dict = field(default_factory=dict)
    kind: str = "bool"

    def T(self) -> "Mat":
        return Mat(self.ncols, self.nrows, {(j, i): v for (i, j), v in self.e.items()}, self.kind)


@dataclass
class Vec:
    n: int
    e: dict = field(default_factory=dict)
    kind: str = "bool"


def _val(x, kind):
    return 1 if kind == "bool" else x


def _cast(x, kind):
    """A value stored in a container of `kind`: int32 keeps the residue
    modulo 2^32 in [-2^31, 2^31) (from fp64, the truncated integer first);
    every other kind keeps the value as it is."""
    if kind != "int32":
        return x
    if isinstance(x, AnyOf):
        return AnyOf({_cast(v, kind) for v in x.c})
    return ((int(x) + 2 ** 31) % 2 ** 32) - 2 ** 31


# Semirings of Table II restricted to the four on the path.  Each is
# (name, multiply(a, b, k), add-monoid, output kind given A's kind).
def _mult(semiring, a, b, k):
    if semiring == "plus.pair":
        return 1
    if semiring == "any.secondi":
        return k
    if semiring == "plus.first":
        return a
    if semiring == "min.plus":
        return float(a) + float(b)
    raise ValueError(semiring)


def _out_kind(semiring, akind):
    if semiring in ("plus.pair", "any.secondi"):
        return "int64"
    if semiring == "plus.first":
        return "int64" if akind == "bool" else akind
    if semiring == "min.plus":
        return "fp64"
    raise ValueError(semiring)


def _reduce_terms(semiring, terms, deterministic):
    """Combine the products, taken in ascending k order."""
    if semiring in ("plus.pair", "plus.first"):
        s = terms[0]
        for t in terms[1:]:
            s = s + t
        return s
    if semiring == "min.plus":
        s = terms[0]
        for t in terms[1:]:
            s = t if t < s else s
        return s
    if semiring == "any.secondi":
        return min(terms) if deterministic or len(set(terms)) == 1 else AnyOf(terms)
    raise ValueError(semiring)


_BINOPS = {
    "plus": lambda c, t: c + t,
    "min": lambda c, t: t if t < c else c,
    "first": lambda c, t: c,
    "second": lambda c, t: t,
    "times": lambda c, t: c * t,
    "div": lambda c, t: c / t,
    "any": lambda c, t: c,
}


def _mask_fn(M, comp, struct, shape_vec=False):
    if M is None:
        return (lambda key: False) if comp else (lambda key: True)

    def f(key):
        present = key in M.e
        on = present and (struct or M.kind == "bool" or _truthy(M.e[key]))
        return (not on) if comp else on

    return f


def _truthy(v):
    if isinstance(v, AnyOf):
        raise ValueError("a valued mask needs concrete values")
    return v != 0


def _write(Cold: dict, T: dict, mask, accum, replace, kind=None):
    """Mask / accumulate / replace step shared by every operation; T's
    values are first stored in the output's kind."""
    T = {key: _cast(t, kind) for key, t in T.items()}
    if accum is None:
        Z = dict(T)
    else:
        op = _BINOPS[accum]
        Z = dict(Cold)
        for key, t in T.items():
            Z[key] = _cast(_lift(op, Cold[key], t), kind) if key in Cold else t
    out = {}
    for key in set(Cold) | set(Z):
        if mask(key):
            if key in Z:
                out[key] = Z[key]
        elif not replace and key in Cold:
            out[key] = Cold[key]
    return out


def product(semiring, A: Mat, B: Mat, deterministic=False, allowed=None) -> dict:
    """T = A plus-times B over `semiring`, dense brute force; `allowed(i, j)`
    may skip positions the mask will discard anyway (it does not change the
    result)."""
    T = {}
    for i in range(A.nrows):
        for j in range(B.ncols):
            if allowed is not None and not allowed((i, j)):
                continue
            terms = []
            for k in range(A.ncols):
                if (i, k) in A.e and (k, j) in B.e:
                    terms.append(_mult(semiring, _val(A.e[(i, k)], A.kind),
                                       _val(B.e[(k, j)], B.kind), k))
            if terms:
                T[(i, j)] = _reduce_terms(semiring, terms, deterministic)
    return T


def mxm(C: Mat, M, accum, semiring, A: Mat, B: Mat, *, comp=False, struct=False,
        replace=False, tran0=False, tran1=False, deterministic=False) -> Mat:
    """C<M> accum= A' semiring B'  (Table I, mxm)."""
    A2 = A.T() if tran0 else A
    B2 = B.T() if tran1 else B
    if A2.ncols != B2.nrows or (C.nrows, C.ncols) != (A2.nrows, B2.ncols):
        raise ValueError("dimension mismatch")
    if M is not None and (M.nrows, M.ncols) != (C.nrows, C.ncols):
        raise ValueError("mask dimension mismatch")
    mask = _mask_fn(M, comp, struct)
    T = product(semiring, A2, B2, deterministic)
    tk = _out_kind(semiring, A2.kind)
    T = {key: _cast(t, tk) for key, t in T.items()}
    return Mat(C.nrows, C.ncols, _write(C.e, T, mask, accum, replace, C.kind), C.kind)


def _row(v: Vec) -> Mat:
    return Mat(1, v.n, {(0, i): x for i, x in v.e.items()}, v.kind)


def vxm(w: Vec, m, accum, semiring, u: Vec, A: Mat, *, comp=False, struct=False,
        replace=False, tran1=False, deterministic=False) -> Vec:
    """w'<m'> accum= u' semiring A'  (Table I, vxm; with tran1 it is the
    pull form A plus-times u of mxv)."""
    Wm = _row(w)
    Mm = None if m is None else _row(m)
    R = mxm(Wm, Mm, accum, semiring, _row(u), A, comp=comp, struct=struct,
            replace=replace, tran1=tran1, deterministic=deterministic)
    return Vec(w.n, {j: x for (_, j), x in R.e.items()}, w.kind)


def ewise_add(C: Mat, M, accum, op, A: Mat, B: Mat, *, comp=False, struct=False,
              replace=False) -> Mat:
    """C<M> accum= A op-union B."""
    f = _BINOPS[op]
    T = {}
    for key in set(A.e) | set(B.e):
        if key in A.e and key in B.e:
            T[key] = _lift(f, _val(A.e[key], A.kind), _val(B.e[key], B.kind))
        elif key in A.e:
            T[key] = _val(A.e[key], A.kind)
        else:
            T[key] = _val(B.e[key], B.kind)
    mask = _mask_fn(M, comp, struct)
    return Mat(C.nrows, C.ncols, _write(C.e, T, mask, accum, replace, C.kind), C.kind)


def ewise_mult(C: Mat, M, accum, op, A: Mat, B: Mat, *, comp=False, struct=False,
               replace=False) -> Mat:
    """C<M> accum= A op-intersection B."""
    f = _BINOPS[op]
    T = {key: _lift(f, _val(A.e[key], A.kind), _val(B.e[key], B.kind))
         for key in set(A.e) & set(B.e)}
    mask = _mask_fn(M, comp, struct)
    return Mat(C.nrows, C.ncols, _write(C.e, T, mask, accum, replace, C.kind), C.kind)


def assign_vector(w: Vec, m, accum, u: Vec, *, comp=False, struct=False, replace=False) -> Vec:
    """w<m>(:) accum= u."""
    mask = _mask_fn(m, comp, struct)
    T = {i: _val(x, u.kind) for i, x in u.e.items()}
    return Vec(w.n, _write(w.e, T, mask, accum, replace, w.kind), w.kind)


def assign_scalar(w: Vec, m, accum, s, *, comp=False, struct=False, replace=False) -> Vec:
    """w<m>(:) accum= s  (every position receives s)."""
    mask = _mask_fn(m, comp, struct)
    T = {i: s for i in range(w.n)}
    return Vec(w.n, _write(w.e, T, mask, accum, replace, w.kind), w.kind)


def reduce_scalar(A, monoid):
    """Reduce every entry to one scalar in row-major index order; None when
    there is no entry."""
    items = sorted(A.e.items())
    kind = A.kind
    vals = [_val(v, kind) for _, v in items]
    if not vals:
        return None
    s = vals[0]
    for v in vals[1:]:
        s = s + v if monoid == "plus" else (v if v < s else s)
    return _cast(s, kind)


def reduce_rows(w: Vec, m, accum, monoid, A: Mat, *, tran0=False, comp=False,
                struct=False, replace=False) -> Vec:
    """w<m> accum= reduce of each row of A' (empty rows give no entry)."""
    A2 = A.T() if tran0 else A
    T = {}
    for i in range(A2.nrows):
        vals = [_val(A2.e[(i, j)], A2.kind) for j in range(A2.ncols) if (i, j) in A2.e]
        if vals:
            s = vals[0]
            for v in vals[1:]:
                s = s + v if monoid == "plus" else (v if v < s else s)
            T[i] = _cast(s, A2.kind)
    mask = _mask_fn(m, comp, struct)
    return Vec(w.n, _write(w.e, T, mask, accum, replace, w.kind), w.kind)


def strictly_lower(A: Mat) -> Mat:
    """select with f(i, j) = j < i (Table I, select)."""
    return Mat(A.nrows, A.ncols, {k: v for k, v in A.e.items() if k[1] < k[0]}, A.kind)


def matches(got, want, rtol=0.0) -> bool:
    """got (a concrete value) is admissible for want (a value or AnyOf)."""
    if isinstance(want, AnyOf):
        return any(matches(got, w, rtol) for w in want.c)
    if isinstance(want, float) or isinstance(got, float):
        if math.isinf(want) or math.isinf(got):
            return want == got
        return abs(float(got) - float(want)) <= rtol * abs(float(want))
    return got == want
