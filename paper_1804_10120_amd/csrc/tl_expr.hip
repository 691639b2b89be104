// Kernels of the paper's benchmark expressions (Sec. 5.1) for gfx950: the
// streaming template of tl_stream.hpp over the bodies of tl_expr_ops.hpp.
// Kept in a translation unit of its own so that the library builds in
// parallel.
#include <hip/hip_runtime.h>

#include "tl_expr_ops.hpp"
#include "tl_internal.hpp"
#include "tl_stream.hpp"

namespace tl {

#define TL_EXPR_OPS(X)                                                                   \
  X(0, OpAssign<1>) X(1, OpAssign<2>) X(2, OpAssign<3>) X(3, OpAdd<2>) X(4, OpAdd<3>)     \
  X(5, OpAdd<4>) X(6, OpMult<2>) X(7, OpMult<3>) X(8, OpMult4) X(9, OpContract<1>)      \
  X(10, OpContract<2>) X(11, OpContract<3>) X(12, OpKij)

hipError_t launch_expr(int id, const Resolved& r, const KArgs& a, int64_t n, hipStream_t s) {
  switch (id) {
#define TL_EXPR(I, OP) \
  case I: return launch_op<OP>(r, a, n, s);
    TL_EXPR_OPS(TL_EXPR)
#undef TL_EXPR
    default: return hipErrorInvalidValue;
  }
}

const void* expr_address(int id, const Resolved& r) {
  switch (id) {
#define TL_EXPR(I, OP) \
  case I: return ptr_op<OP>(r);
    TL_EXPR_OPS(TL_EXPR)
#undef TL_EXPR
    default: return nullptr;
  }
}

int expr_ppt(int id, int ppt) {
  switch (id) {
#define TL_EXPR(I, OP) \
  case I: return op_ppt<OP>(ppt);
    TL_EXPR_OPS(TL_EXPR)
#undef TL_EXPR
    default: return ppt;
  }
}

}  // namespace tl
