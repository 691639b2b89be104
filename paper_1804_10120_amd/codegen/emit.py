"""HIP emitter: a Program becomes a streaming per-point body for gfx950, a
C-ABI entry point ``tlg_<name>``, a header declaration and a manifest entry.

The body evaluates the statements with every index substituted and every sum
unrolled (straight-line FP64 code; the compiler shares common
subexpressions), keeps temporaries in registers and stores each output
component as soon as it is computed.  Before unrolling, factors that do not
depend on a sum's index are moved out of the sum, so a chain of contractions
is evaluated one index at a time (the partial sums are shared between the
output components that need them); the output components are then visited
with the indices of the innermost factors outermost, so that the partial sums
of one slice are used up before the next slice's are formed.  A body with few
inputs loads them all first (so they are in flight together); one with many
loads each input at its first use and keeps the compiler from moving work
between slices, so only one slice's inputs are live at a time.  The body runs
through the library's streaming template, so it gets the same launch shapes,
non-temporal accesses and XCD order as the hand-written kernels.
"""
from __future__ import annotations

from .dsl import Bin, CodegenError, Const, Neg, Program, Ref, SumExpr


def render(e) -> str:
    """Index notation of an expression (for documentation)."""
    if isinstance(e, Const):
        return repr(e.value)
    if isinstance(e, Ref):
        return f"{e.tensor.name}(" + ",".join(repr(a) for a in e.args) + ")"
    if isinstance(e, Bin):
        return f"({render(e.a)} {e.op} {render(e.b)})"
    if isinstance(e, Neg):
        return f"-{render(e.a)}"
    if isinstance(e, SumExpr):
        return f"Sum({e.index}, {render(e.body)})"
    raise CodegenError(repr(e))


def statement_text(st) -> str:
    return f"{render(st.lhs)} = {render(st.rhs)}"


def tensor_text(t) -> str:
    dims = "x".join(str(d) for d in t.dims) or "scalar"
    sym = "".join(f", symmetric in slots {p},{q}" for p, q in t.sym)
    return f"{t.name} [{t.ncomp}] ({dims}{sym})"


# Programs with more input components than WIDE_INPUTS run in blocks of at
# most WIDE_MAX_BLOCK threads.  Programs with more than LAZY_INPUTS load each
# input at its first use, slice by slice, instead of all inputs first.
WIDE_INPUTS = 100
WIDE_MAX_BLOCK = 256
LAZY_INPUTS = 64


def _factors(e):
    if isinstance(e, Bin) and e.op == "*":
        return _factors(e.a) + _factors(e.b)
    return [e]


def _product(fs):
    out = fs[0]
    for f in fs[1:]:
        out = Bin("*", out, f)
    return out


def _depends(e, index) -> bool:
    return any(x is index for x in e.free())


def factor_sums(e):
    """The expression with every factor that does not depend on a sum's index
    moved out of that sum (innermost sums first): Sum(m, Sum(n, B(i,m) C(j,n)
    E(m,n,k))) becomes Sum(m, B(i,m) Sum(n, C(j,n) E(m,n,k))).  Exact algebra;
    only the rounding order changes."""
    if isinstance(e, SumExpr):
        fs = _factors(factor_sums(e.body))
        indep = [f for f in fs if not _depends(f, e.index)]
        dep = [f for f in fs if _depends(f, e.index)]
        inner = SumExpr(e.index, _product(dep))
        return _product(indep + [inner]) if indep else inner
    if isinstance(e, Bin):
        return Bin(e.op, factor_sums(e.a), factor_sums(e.b))
    if isinstance(e, Neg):
        return Neg(factor_sums(e.a))
    return e


def index_order(lhs_free, rhs):
    """The left-hand indices, outermost first: those met deepest inside the
    sums of the (factored) right-hand side first, among equals those of the
    larger tensor, then in written order."""
    depth, size = {}, {}

    def walk(e, d):
        if isinstance(e, Ref):
            for a in e.free():
                if depth.get(id(a), -1) < d or (depth[id(a)] == d and
                                                size[id(a)] < e.tensor.ncomp):
                    depth[id(a)], size[id(a)] = d, e.tensor.ncomp
        elif isinstance(e, Bin):
            walk(e.a, d)
            walk(e.b, d)
        elif isinstance(e, Neg):
            walk(e.a, d)
        elif isinstance(e, SumExpr):
            walk(e.body, d + 1)

    walk(rhs, 0)
    pos = {id(x): k for k, x in enumerate(lhs_free)}
    return sorted(lhs_free, key=lambda x: (-depth.get(id(x), 0), -size.get(id(x), 0),
                                           pos[id(x)]))


class _Emitter:
    def __init__(self, prog: Program):
        prog.check()
        self.p = prog
        self.ins = prog.inputs
        self.outs = prog.outputs
        self.fin = {t: f for f, t in enumerate(self.ins)}
        self.fout = {t: f for f, t in enumerate(self.outs)}
        self.loaded = {}         # (field, comp) -> variable
        self.pending = []        # loads referenced since the last statement was emitted
        self.written = set()     # (field, comp) of outputs with a value
        self.temp_written = set()  # (temporary, comp) with a value
        self.lazy = sum(t.ncomp for t in self.ins) > LAZY_INPUTS

    def ref(self, e: Ref, env) -> str:
        t = e.tensor
        c = t.comp(e.resolve(env))
        if t in self.p.temps:
            if (t, c) not in self.temp_written:
                raise CodegenError(f"temporary {t.name}[{c}] is read before it is written")
            return f"t_{t.name}[{c}]"
        if t in self.fin:
            key = (self.fin[t], c)
            if key not in self.loaded:
                self.loaded[key] = f"x{key[0]}_{c}"
                self.pending.append(key)
            return self.loaded[key]
        f = self.fout[t]
        if (f, c) not in self.written:
            raise CodegenError(f"{t.name}[{c}] is read before it is written")
        return f"o{f}_{c}"

    def expr(self, e, env) -> str:
        if isinstance(e, Const):
            return repr(e.value)
        if isinstance(e, Ref):
            return self.ref(e, env)
        if isinstance(e, Bin):
            return f"({self.expr(e.a, env)} {e.op} {self.expr(e.b, env)})"
        if isinstance(e, Neg):
            return f"(-{self.expr(e.a, env)})"
        if isinstance(e, SumExpr):
            return "(" + " + ".join(self.expr(e.body, {**env, e.index: v})
                                    for v in range(e.index.dim)) + ")"
        raise CodegenError(repr(e))

    def _flush_loads(self, out):
        for f, c in self.pending:
            out.append(f"    const double {self.loaded[(f, c)]} = ld({f}, {c});")
        self.pending = []

    def _emit(self, st, items, stmts, declared, order):
        """The components ``items`` of statement ``st``, in order."""
        t = st.lhs.tensor
        rhs_f = factor_sums(st.rhs)
        outer = None
        for c, env in items:
            if self.lazy and order:
                if outer is not None and env[order[0]] != outer:
                    # the next slice: nothing moves across this point
                    stmts.append("    __builtin_amdgcn_sched_barrier(0);")
                outer = env[order[0]]
            rhs = self.expr(rhs_f, env)
            if self.lazy:
                self._flush_loads(stmts)
            if t in self.p.temps:
                self.temp_written.add((t, c))
                stmts.append(f"    t_{t.name}[{c}] = {rhs};")
            else:
                f = self.fout[t]
                var = f"o{f}_{c}"
                decl = "" if (f, c) in declared else "double "
                declared.add((f, c))
                self.written.add((f, c))
                stmts.append(f"    {decl}{var} = {rhs};")
                stmts.append(f"    st({f}, {c}, {var});")

    def body(self) -> str:
        lines = []
        for t in self.p.temps:
            lines.append(f"    double t_{t.name}[{t.ncomp}];")
        stmts = []
        declared = set()
        plans = []
        for st in self.p.statements:
            order = index_order(st.lhs.free(), factor_sums(st.rhs))
            if self.p.fused is not None:   # the fused index outermost
                order = [self.p.fused] + [x for x in order if x is not self.p.fused]
            todo = sorted(st.assignments(), key=lambda ce: tuple(ce[1][x] for x in order))
            plans.append((st, order, todo))
        if self.p.fused is None:
            for st, order, todo in plans:
                stmts.append(f"    // {statement_text(st)}")
                self._emit(st, todo, stmts, declared, order)
        else:
            x = self.p.fused
            for st, _, _ in plans:
                stmts.append(f"    // {statement_text(st)}")
            stmts.append(f"    // slice by slice in {x}")
            for v in range(x.dim):
                if v:
                    stmts.append("    __builtin_amdgcn_sched_barrier(0);")
                for st, order, todo in plans:
                    self._emit(st, [ce for ce in todo if ce[1][x] == v], stmts, declared,
                               order[1:])
        if self.lazy:
            return "\n".join(lines + stmts)
        loads = [f"    const double {v} = ld({f}, {c});"
                 for (f, c), v in sorted(self.loaded.items())]
        return "\n".join(lines + loads + stmts)

    def struct(self) -> str:
        p = self.p
        body = self.body()
        fin = ", ".join(str(t.ncomp) for t in self.ins)
        fout = ", ".join(str(t.ncomp) for t in self.outs)
        nin = sum(t.ncomp for t in self.ins)
        cap = (f"\n  static constexpr int kMaxBlock = {WIDE_MAX_BLOCK};  // more than "
               f"{WIDE_INPUTS} inputs" if nin > WIDE_INPUTS else "")
        return f"""// {p.name}: {p.doc}
struct Gen_{p.name} {{
  static constexpr bool kStream = true;{cap}
  static constexpr int NF_IN = {len(self.ins)}, NF_OUT = {len(self.outs)};
  static constexpr int fin[NF_IN] = {{{fin}}};
  static constexpr int fout[NF_OUT] = {{{fout}}};
  static constexpr int NIN = {sum(t.ncomp for t in self.ins)}, NOUT = {sum(t.ncomp for t in self.outs)};
  template <class L, class S>
  __device__ static inline void stream(L&& ld, S&& st) {{
{body}
  }}
}};
"""

    def signature(self) -> str:
        return (f"tl_status tlg_{self.p.name}(int64_t n, const tl_cfield* in, int32_t nin, "
                f"const tl_field* out, int32_t nout, void* stream, const tl_tune* tune)")

    def entry(self) -> str:
        p = self.p
        fin = ", ".join(str(t.ncomp) for t in self.ins)
        fout = ", ".join(str(t.ncomp) for t in self.outs)
        return f"""{self.signature()} {{
  static const int32_t kIn[] = {{{fin}}};
  static const int32_t kOut[] = {{{fout}}};
  return tl::run_generated("{p.name}", n, in, nin, kIn, {len(self.ins)}, out, nout, kOut,
                           {len(self.outs)}, stream, tune, &tl::launch_op<tl::Gen_{p.name}>);
}}
"""

    def declaration(self) -> str:
        p = self.p
        lines = [f"/* {p.name}: {p.doc}"]
        for st in p.statements:
            lines.append(f" *   {statement_text(st)}")
        if p.temps:
            lines.append(" * in registers only: " + ", ".join(sorted(t.name for t in p.temps)))
        lines.append(" * in:  " + "; ".join(tensor_text(t) for t in self.ins))
        lines.append(" * out: " + "; ".join(tensor_text(t) for t in self.outs))
        lines.append(f" * stored elements read + written per point (BW_eff N_e): {p.elements()} */")
        return "\n".join(lines) + "\n" + self.signature() + ";\n"

    def manifest(self) -> dict:
        p = self.p
        return {"name": p.name, "doc": p.doc,
                "statements": [statement_text(st) for st in p.statements],
                "inputs": [{"name": t.name, "ncomp": t.ncomp, "dims": list(t.dims),
                            "sym": [list(s) for s in t.sym]} for t in self.ins],
                "outputs": [{"name": t.name, "ncomp": t.ncomp, "dims": list(t.dims),
                             "sym": [list(s) for s in t.sym]} for t in self.outs],
                "elements": p.elements()}


HEADER_TOP = """/*
 * tl_generated.h -- entry points generated from index notation
 * (paper_1804_10120_amd/codegen; regenerate with
 * `python -m paper_1804_10120_amd.codegen`, do not edit by hand).
 *
 * The code generator is this library's counterpart of the paper's automatic
 * code generation (Sec. 3): tensor expressions written in index notation,
 * with symmetric slots, fixed and offset indices and explicit sums (Sec. 2.3 -
 * 2.5), become straight-line FP64 kernels for gfx950 that run through the same
 * streaming launch machinery as the hand-written kernels of tl.h.
 *
 * Calling convention of every tlg_<name>:
 *   in[0..nin-1]   the input fields, in the order listed (tl_cfield, [C][ld]);
 *   out[0..nout-1] the output fields, in the order listed (tl_field);
 *   nin, nout must equal the counts listed; components of a tensor are its
 *   index tuples in lexicographic order, keeping only first <= second within
 *   each symmetric slot pair (so s(i,j) = 00 01 02 11 12 22 for 3x3);
 *   a component of a symmetric left-hand side is evaluated with the first
 *   index of the pair >= the second, the member the paper's loops for a
 *   symmetric left-hand side visit (Sec. 2.4, Sec. 4), and stored in its slot;
 *   an output component that no statement writes is left untouched.
 * Ownership, execution (asynchronous on `stream`), tuning and errors are as
 * for the entry points of tl.h (TL_ERR_INVALID for a wrong nin or nout).
 */
#ifndef TL_GENERATED_H
#define TL_GENERATED_H

#include "tl.h"

#ifdef __cplusplus
extern "C" {
#endif

"""

HEADER_BOTTOM = """
#ifdef __cplusplus
}
#endif

#endif /* TL_GENERATED_H */
"""

SOURCE_TOP = """// Generated from index notation by paper_1804_10120_amd/codegen (regenerate
// with `python -m paper_1804_10120_amd.codegen`, do not edit by hand).
// Streaming per-point bodies for gfx950 and their C-ABI entry points; see
// include/tl_generated.h for the expressions.
#include <hip/hip_runtime.h>

#include "../../../include/tl_generated.h"
#include "../tl_internal.hpp"
#include "../tl_stream.hpp"

namespace tl {

"""


def generate(programs):
    """(HIP source, header, manifest) for a list of programs."""
    names = [p.name for p in programs]
    if len(set(names)) != len(names):
        raise CodegenError("program names must be unique")
    ems = [_Emitter(p) for p in programs]
    structs = "\n".join(e.struct() for e in ems)
    entries = "\n".join(e.entry() for e in ems)
    src = SOURCE_TOP + structs + "\n}  // namespace tl\n\nextern \"C\" {\n\n" + entries + \
        "\n}  // extern \"C\"\n"
    hdr = HEADER_TOP + "\n".join(e.declaration() for e in ems) + HEADER_BOTTOM
    man = {"programs": [e.manifest() for e in ems]}
    return src, hdr, man
