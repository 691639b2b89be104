"""Index-notation front end: tensors, indices, expressions, programs.

The expressions are the ones of the paper's expression templates (Sec. 2.3 -
2.5): indexed tensors with spatial (dimension 3) or spacetime (dimension 4)
indices, fixed indices (an integer in an index slot) and offset indices
(``i + 1``), symmetric index pairs, sums, differences, products, scalar
constants and explicit contractions ``Sum(l, ...)`` -- as in the paper, an
index repeated inside a product must be summed explicitly.  A program is a
sequence of assignments; tensors that are written and not declared temporary
are outputs, tensors only read are inputs, temporaries live in registers.

Component storage: a tensor's independent components are its index tuples
in lexicographic order, keeping for every symmetric slot pair only the tuples
with the first index <= the second.  This reproduces the layouts of the
hand-written kernels (s(i,j) = 00 01 02 11 12 22; derivative-first
d_k g_ij at k*6 + s(i,j); Gamma^i_jk at i*6 + s(j,k); row-major
non-symmetric tensors).
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass


class CodegenError(ValueError):
    """An expression that violates the index rules."""


class Index:
    """A free or summed tensor index ranging over 0 .. dim-1."""

    def __init__(self, name: str, dim: int = 3):
        if dim not in (3, 4):
            raise CodegenError(f"index {name}: dimension {dim} (3 or 4 supported)")
        self.name, self.dim = name, dim

    def __add__(self, k: int) -> "Offset":
        return Offset(self, int(k))

    def __repr__(self):
        return self.name


@dataclass(frozen=True)
class Offset:
    """An index shifted by a constant: slot value = index value + k."""
    index: Index
    k: int

    def __repr__(self):
        return f"{self.index.name}+{self.k}"


def indices(names: str, dim: int = 3):
    """``i, j, k = indices("i j k")`` (dimension 3) or ``indices("a b", 4)``."""
    return tuple(Index(n, dim) for n in names.split())


class Tensor:
    """A tensor field: one dimension per slot and disjoint symmetric slot pairs."""

    def __init__(self, name: str, dims=(), sym=()):
        self.name = name
        self.dims = tuple(int(d) for d in dims)
        self.sym = tuple(tuple(sorted(p)) for p in sym)
        used = [s for p in self.sym for s in p]
        if len(used) != len(set(used)) or any(not 0 <= s < len(self.dims) for s in used):
            raise CodegenError(f"{name}: symmetric pairs must be disjoint slot pairs")
        for p, q in self.sym:
            if self.dims[p] != self.dims[q]:
                raise CodegenError(f"{name}: symmetric slots {p},{q} differ in dimension")
        self.components = [t for t in itertools.product(*[range(d) for d in self.dims])
                           if all(t[p] <= t[q] for p, q in self.sym)]
        self._index = {t: c for c, t in enumerate(self.components)}

    @property
    def rank(self):
        return len(self.dims)

    @property
    def ncomp(self):
        return len(self.components)

    def canonical(self, t):
        t = list(t)
        for p, q in self.sym:
            if t[p] > t[q]:
                t[p], t[q] = t[q], t[p]
        return tuple(t)

    def comp(self, t):
        """Storage index of the component with index values ``t``."""
        t = tuple(t)
        if len(t) != self.rank or any(not 0 <= v < d for v, d in zip(t, self.dims)):
            raise CodegenError(f"{self.name}{list(t)} is out of range {self.dims}")
        return self._index[self.canonical(t)]

    def __getitem__(self, args):
        if not isinstance(args, tuple):
            args = (args,)
        if len(args) != self.rank:
            raise CodegenError(f"{self.name} has {self.rank} slots, got {len(args)} indices")
        for s, a in enumerate(args):
            if isinstance(a, Index):
                if a.dim > self.dims[s]:
                    raise CodegenError(f"{self.name} slot {s}: index {a} ranges over {a.dim}, "
                                       f"slot over {self.dims[s]}")
            elif isinstance(a, Offset):
                if a.index.dim + a.k > self.dims[s] or a.k < 0:
                    raise CodegenError(f"{self.name} slot {s}: {a} leaves 0..{self.dims[s] - 1}")
            elif isinstance(a, int):
                if not 0 <= a < self.dims[s]:
                    raise CodegenError(f"{self.name} slot {s}: fixed index {a} out of range")
            else:
                raise CodegenError(f"{self.name}: bad index {a!r}")
        return Ref(self, args)

    def __repr__(self):
        return self.name


# ---------------------------------------------------------------- expressions

class Expr:
    def __add__(self, o):
        return Bin("+", self, _wrap(o))

    def __radd__(self, o):
        return Bin("+", _wrap(o), self)

    def __sub__(self, o):
        return Bin("-", self, _wrap(o))

    def __rsub__(self, o):
        return Bin("-", _wrap(o), self)

    def __mul__(self, o):
        return Bin("*", self, _wrap(o))

    def __rmul__(self, o):
        return Bin("*", _wrap(o), self)

    def __neg__(self):
        return Neg(self)


def _wrap(x):
    if isinstance(x, Expr):
        return x
    if isinstance(x, (int, float)):
        return Const(float(x))
    raise CodegenError(f"cannot use {x!r} in an expression")


@dataclass(eq=False)
class Const(Expr):
    value: float

    def free(self):
        return []


@dataclass(eq=False)
class Ref(Expr):
    tensor: Tensor
    args: tuple

    def free(self):
        out = []
        for a in self.args:
            if isinstance(a, Index):
                out.append(a)
            elif isinstance(a, Offset):
                out.append(a.index)
        return out

    def resolve(self, env):
        vals = []
        for a in self.args:
            if isinstance(a, Index):
                vals.append(env[a])
            elif isinstance(a, Offset):
                vals.append(env[a.index] + a.k)
            else:
                vals.append(a)
        return tuple(vals)


@dataclass(eq=False)
class Bin(Expr):
    op: str
    a: Expr
    b: Expr

    def free(self):
        fa, fb = self.a.free(), self.b.free()
        if self.op == "*":
            return fa + fb
        if _multiset(fa) != _multiset(fb):
            raise CodegenError(f"operands of '{self.op}' have different free indices "
                               f"{fa} and {fb}")
        return fa


@dataclass(eq=False)
class Neg(Expr):
    a: Expr

    def free(self):
        return self.a.free()


@dataclass(eq=False)
class SumExpr(Expr):
    index: Index
    body: Expr

    def free(self):
        f = self.body.free()
        if self.index not in f:
            raise CodegenError(f"Sum over {self.index}, which does not appear in its body")
        return [x for x in f if x is not self.index]


def Sum(index: Index, body) -> SumExpr:
    """Explicit contraction over ``index`` (the paper's ``Sum``)."""
    return SumExpr(index, _wrap(body))


def _multiset(xs):
    out = {}
    for x in xs:
        out[id(x)] = out.get(id(x), 0) + 1
    return out


# ---------------------------------------------------------------- programs

@dataclass
class Statement:
    lhs: Ref
    rhs: Expr

    def check(self):
        lf = self.lhs.free()
        if len({id(x) for x in lf}) != len(lf):
            raise CodegenError(f"{self.lhs.tensor}: an index repeats on the left-hand side")
        rf = self.rhs.free()
        if len({id(x) for x in rf}) != len(rf):
            dup = [x for x in rf if rf.count(x) > 1]
            raise CodegenError(f"index {dup[0]} repeats outside a Sum (write the sum "
                               "explicitly)")
        if {id(x) for x in lf} != {id(x) for x in rf} and rf:
            raise CodegenError(f"{self.lhs.tensor}: left-hand indices {lf} differ from the "
                               f"right-hand side's {rf}")
        if not rf and lf:
            # a right-hand side without free indices broadcasts over the left-hand side
            pass

    def assignments(self):
        """(LHS storage component, index environment) for every component the
        statement writes, in the order the components are first reached with
        the free LHS indices running lexicographically.  A component reached
        by several index tuples (both slots of a symmetric pair free) is
        written once, evaluated at the tuple whose first slot of each
        symmetric pair is >= the second: the paper's loops for a symmetric
        left-hand side start the first index of the pair at the value of the
        second (the tensor-index loop of Sec. 2.4; the generated C loop and
        CUDA kernel of the rank-2 contraction example, Sec. 4).  When the
        right-hand side is not symmetric this decides which of C_ab and C_ba
        is stored."""
        lf = self.lhs.free()
        sym = self.lhs.tensor.sym
        where = {}
        out = []
        for vals in itertools.product(*[range(x.dim) for x in lf]):
            env = dict(zip(lf, vals))
            t = self.lhs.resolve(env)
            c = self.lhs.tensor.comp(t)
            if c not in where:
                where[c] = len(out)
                out.append((c, env))
            elif all(t[p] >= t[q] for p, q in sym):
                out[where[c]] = (c, env)
        return out


class Program:
    """A named sequence of assignments compiled into one kernel."""

    def __init__(self, name: str, doc: str = ""):
        if not name.isidentifier():
            raise CodegenError(f"program name {name!r} is not an identifier")
        self.name, self.doc = name, doc
        self.statements = []
        self.temps = []
        self.fused = None
        self.arg_order = None

    def input_order(self, *tensors):
        """Pass the inputs in this order (default: order of first appearance),
        e.g. to keep an expression's written order once it is split into
        several statements."""
        self.arg_order = list(tensors)
        return self

    def fuse(self, index: Index):
        """Evaluate the statements slice by slice in ``index`` (a free index
        of every left-hand side): all statements at index value 0, then at 1,
        ...  A statement may then read a temporary only at the slice being
        evaluated, so each slice's temporaries are used up before the next
        slice's are formed (the generator rejects a read of a temporary
        component not yet written)."""
        if not isinstance(index, Index):
            raise CodegenError("fuse() takes an index")
        self.fused = index
        return self

    def temp(self, *tensors):
        """Declare tensors that stay in registers (never read or written in memory)."""
        for t in tensors:
            if t not in self.temps:
                self.temps.append(t)
        return self

    def let(self, lhs: Ref, rhs):
        if not isinstance(lhs, Ref):
            raise CodegenError("the left-hand side must be an indexed tensor")
        st = Statement(lhs, _wrap(rhs))
        st.check()
        self.statements.append(st)
        return self

    # tensor roles, in order of first appearance
    def _order(self):
        seen, out = set(), []

        def walk(e):
            if isinstance(e, Ref):
                if e.tensor not in seen:
                    seen.add(e.tensor)
                    out.append(e.tensor)
            elif isinstance(e, Bin):
                walk(e.a)
                walk(e.b)
            elif isinstance(e, (Neg,)):
                walk(e.a)
            elif isinstance(e, SumExpr):
                walk(e.body)

        for st in self.statements:
            walk(st.rhs)
            walk(st.lhs)
        return out

    @property
    def outputs(self):
        written = {st.lhs.tensor for st in self.statements}
        return [t for t in self._order() if t in written and t not in self.temps]

    @property
    def inputs(self):
        written = {st.lhs.tensor for st in self.statements}
        found = [t for t in self._order() if t not in written]
        if self.arg_order is None:
            return found
        if set(self.arg_order) != set(found) or len(self.arg_order) != len(found):
            raise CodegenError(f"{self.name}: input_order {self.arg_order} does not name the "
                               f"inputs {found}")
        return list(self.arg_order)

    def check(self):
        if self.fused is not None:
            for st in self.statements:
                if not any(x is self.fused for x in st.lhs.free()):
                    raise CodegenError(f"{self.name}: fused index {self.fused} is not free on "
                                       f"the left-hand side of {st.lhs.tensor}")
        written = set()
        for st in self.statements:
            for t in _reads(st.rhs):
                if t in self.temps and t not in written:
                    raise CodegenError(f"temporary {t} is read before it is written")
            written.add(st.lhs.tensor)
        for t in self.temps:
            if t not in written:
                raise CodegenError(f"temporary {t} is never written")
        if not self.outputs:
            raise CodegenError(f"{self.name}: nothing is written to memory")
        return self

    def elements(self):
        """Distinct stored components read and written per point: the paper's
        N_e of the effective bandwidth (Sec. 5.1), temporaries excluded."""
        self.check()
        read = {t: set() for t in self.inputs}
        written = {t: set() for t in self.outputs}
        for st in self.statements:
            for c, env in st.assignments():
                if st.lhs.tensor in written:
                    written[st.lhs.tensor].add(c)
                _collect_reads(st.rhs, env, read)
        return sum(len(v) for v in read.values()) + sum(len(v) for v in written.values())


def _reads(e):
    if isinstance(e, Ref):
        return [e.tensor]
    if isinstance(e, Bin):
        return _reads(e.a) + _reads(e.b)
    if isinstance(e, Neg):
        return _reads(e.a)
    if isinstance(e, SumExpr):
        return _reads(e.body)
    return []


def _collect_reads(e, env, read):
    if isinstance(e, Ref):
        if e.tensor in read:
            read[e.tensor].add(e.tensor.comp(e.resolve(env)))
    elif isinstance(e, Bin):
        _collect_reads(e.a, env, read)
        _collect_reads(e.b, env, read)
    elif isinstance(e, Neg):
        _collect_reads(e.a, env, read)
    elif isinstance(e, SumExpr):
        for v in range(e.index.dim):
            _collect_reads(e.body, {**env, e.index: v}, read)
