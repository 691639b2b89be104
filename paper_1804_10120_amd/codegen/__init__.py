"""Index notation -> HIP code generator (the counterpart of the paper's
automatic code generation, Sec. 3)."""
from .dsl import CodegenError, Index, Program, Sum, Tensor, indices
from .emit import generate, render, statement_text

__all__ = ["CodegenError", "Index", "Program", "Sum", "Tensor", "indices", "generate", "render",
           "statement_text"]
