// Internal interface between the C ABI (tl_abi.cpp) and the kernels
// (tl_kernels.hip).  Not installed, not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/tl.h"

namespace tl {

constexpr int kMaxFields = 8;

// Base pointer and leading dimension of each input and output field, in the
// field order of the kernel's per-point body.  A NULL output is skipped.
struct KArgs {
  const double* in[kMaxFields];
  int64_t ldin[kMaxFields];
  double* out[kMaxFields];
  int64_t ldout[kMaxFields];
};

// One subgrid of a batch plan, as stored in device memory.
struct alignas(64) BatchDomain {
  KArgs args;
  int64_t n;
};

// Generic: a body chosen by the caller (the benchmark expressions, the
// bandwidth twins, generated kernels): the fused chain's default shapes, and
// the points per lane settled by the body's stream count (op_ppt).
enum class KernelId { SymInverse, Christoffel, CovDeriv, Dtg, Chain, ChainBwd, ChainBatched,
                      ChainFwdBwd, ChainBwdBatched, Generic };

// A tuning request resolved to one compiled instantiation.
struct Resolved {
  int block = 256;
  int ppt = 1;       // 1, 2 or 4 (4 only for bodies with few component streams)
  bool nt = false;
  bool xcd = false;  // XCD-contiguous tile order (grid is then a multiple of 8)
  int grid_mult = 0;
  int num_cu = 256;
  bool buf = false;  // buffer addressing (every field's extent below 4 GiB)
  int lanes = 1;     // lanes per grid point (tl_christoffel only)
};

inline int64_t grid_size(const Resolved& r, int64_t ntiles) {
  int64_t g = ntiles;
  if (r.grid_mult > 0) {
    const int64_t cap = static_cast<int64_t>(r.grid_mult) * r.num_cu;
    if (g > cap) g = cap;
  }
  if (g > 0x7ffffff0) g = 0x7ffffff0;
  if (g < 1) g = 1;
  if (r.xcd) g = (g + 7) & ~static_cast<int64_t>(7);
  return g;
}

// (reads, writes) shapes of the bandwidth twin: those of the rows, and a copy.
#define TL_TWIN_SHAPES(X) X(1, 1) X(6, 6) X(24, 18) X(30, 9) X(16, 6) X(43, 6) X(40, 43)

hipError_t launch_kernel(KernelId k, const Resolved& r, const KArgs& a, int64_t n, hipStream_t s);
hipError_t launch_twin(int nin, int nout, const Resolved& r, const KArgs& a, int64_t n,
                       hipStream_t s);
const void* kernel_address(KernelId k, const Resolved& r);
// The benchmark expressions (ids as in tl_expr_id of tl.h).
hipError_t launch_expr(int id, const Resolved& r, const KArgs& a, int64_t n, hipStream_t s);
const void* expr_address(int id, const Resolved& r);
// Points per lane expression `id` runs with when `ppt` is requested.
int expr_ppt(int id, int ppt);
// Validation, tuning and launch for a generated entry point: nin/nout and
// the fields' component counts are checked against the expected ones.
typedef hipError_t (*LaunchFn)(const Resolved&, const KArgs&, int64_t, hipStream_t);
tl_status run_generated(const char* name, int64_t n, const tl_cfield* in, int32_t nin,
                        const int32_t* in_ncomp, int32_t nin_expected, const tl_field* out,
                        int32_t nout, const int32_t* out_ncomp, int32_t nout_expected,
                        void* stream, const tl_tune* tune, LaunchFn launch);

hipError_t launch_batched(KernelId k, const Resolved& r, const BatchDomain* doms, const int64_t* start,
                          const int32_t* tile_dom, int64_t ntiles, int64_t grid, int64_t chunk,
                          hipStream_t s);
// The forward batched kernel with its tables written into the library's
// fixed per-device array (tl_noalloc.hip); doms and start are host arrays of
// the plan tables (ndom descriptors, ndom + 1 tile starts).
hipError_t launch_batched_noalloc(const Resolved& r, const BatchDomain* doms, const int64_t* start,
                                  int32_t ndom, int64_t ntiles, int64_t grid, int64_t chunk,
                                  hipStream_t s);
hipError_t launch_copy(const double* src, double* dst, int64_t n, int64_t grid, hipStream_t s);
hipError_t launch_read(const double* src, double* partial, int64_t n, int64_t grid, bool vec,
                       hipStream_t s);
hipError_t launch_write(double* dst, int64_t n, int64_t grid, bool vec, hipStream_t s);
hipError_t launch_christoffel_lanes(const Resolved& r, const KArgs& a, int64_t n, hipStream_t s);

// Registers, scratch and occupancy of one compiled kernel, as the compiler
// reported them when the library was built (the build writes the table).
struct KernelResources {
  int sgprs;           // scalar registers per wave, VCC and other reserved ones included
  int vgprs;           // architected vector registers per lane
  int agprs;           // accumulation registers per lane
  int scratch;         // private (scratch) bytes per lane
  int waves_per_simd;  // occupancy bound from the resources alone
};
// Looks a kernel up by its mangled (or demangled) name; false if unknown.
bool kernel_resources(const char* name, KernelResources* out);

}  // namespace tl
