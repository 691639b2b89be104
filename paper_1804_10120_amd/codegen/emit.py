"""HIP emitter: a Program becomes a streaming per-point body for gfx950, a
C-ABI entry point ``tlg_<name>``, a header declaration and a manifest entry.

The body loads every referenced input component once (all loads first, so
they are in flight together), evaluates the statements with every index
substituted and every sum unrolled (straight-line FP64 code; the compiler
shares common subexpressions), keeps temporaries in registers and stores each
output component as soon as it is computed.  It runs through the library's
streaming template, so it gets the same launch shapes, non-temporal accesses
and XCD order as the hand-written kernels.
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


# Programs with more input components than WIDE_INPUTS keep them all live and
# run in blocks of at most WIDE_MAX_BLOCK threads, which their registers fit.
WIDE_INPUTS = 100
WIDE_MAX_BLOCK = 256


class _Emitter:
    def __init__(self, prog: Program):
        prog.check()
        self.p = prog
        self.ins = prog.inputs
        self.outs = prog.outputs
        self.fin = {t: f for f, t in enumerate(self.ins)}
        self.fout = {t: f for f, t in enumerate(self.outs)}
        self.loaded = {}         # (field, comp) -> variable
        self.written = set()     # (field, comp) of outputs with a value

    def ref(self, e: Ref, env) -> str:
        t = e.tensor
        c = t.comp(e.resolve(env))
        if t in self.p.temps:
            return f"t_{t.name}[{c}]"
        if t in self.fin:
            key = (self.fin[t], c)
            if key not in self.loaded:
                self.loaded[key] = f"x{key[0]}_{c}"
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

    def body(self) -> str:
        lines = []
        for t in self.p.temps:
            lines.append(f"    double t_{t.name}[{t.ncomp}];")
        stmts = []
        declared = set()
        for st in self.p.statements:
            stmts.append(f"    // {statement_text(st)}")
            t = st.lhs.tensor
            for c, env in st.assignments():
                rhs = self.expr(st.rhs, env)
                if t in self.p.temps:
                    stmts.append(f"    t_{t.name}[{c}] = {rhs};")
                else:
                    f = self.fout[t]
                    var = f"o{f}_{c}"
                    decl = "" if (f, c) in declared else "double "
                    declared.add((f, c))
                    self.written.add((f, c))
                    stmts.append(f"    {decl}{var} = {rhs};")
                    stmts.append(f"    st({f}, {c}, {var});")
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
               f"{WIDE_INPUTS} inputs live" if nin > WIDE_INPUTS else "")
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
