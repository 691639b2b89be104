// Kernels of the tensor-expression chain for gfx950 and their launchers:
// the unfused steps, the fused chain and its adjoint (all through the
// streaming template of tl_stream.hpp), the batched kernel over many
// subgrids, the bandwidth twins and the streaming copy.
#include <hip/hip_runtime.h>

#include "tl_device.hpp"
#include "tl_internal.hpp"
#include "tl_stream.hpp"

namespace tl {

// Many subgrids: global tile t belongs to subgrid d = tile_dom[t] and is that
// subgrid's tile t - start[d] (block-uniform loads, so scalar).  Block lb
// walks the contiguous chunk of tiles [lb*chunk, (lb+1)*chunk), so
// consecutive tiles of a block are mostly in the same subgrid and its
// descriptor is fetched again only when the subgrid changes.  With chunk = 1
// and one block per tile this is a plain (non-persistent) launch.  Op is the
// per-point body: the fused chain (OpChain) or its adjoint (OpChainBwd).
template <class Op, int BLOCK, int PPT, bool NT, bool BUF>
__global__ __launch_bounds__(BLOCK) void k_batched(const BatchDomain* __restrict__ doms,
                                                    const int64_t* __restrict__ start,
                                                    const int32_t* __restrict__ tile_dom,
                                                    int64_t ntiles, int64_t chunk, int32_t xcd) {
  const int64_t t0 = logical_block(xcd) * chunk;
  const int64_t t1 = t0 + chunk < ntiles ? t0 + chunk : ntiles;
  int32_t cur = -1;
  KArgs a;
  Bufs<Op> b;
  int64_t n = 0, s0 = 0;
  for (int64_t t = t0; t < t1; ++t) {
    const int32_t d = tile_dom[t];
    if (d != cur) {
      cur = d;
      a = doms[d].args;
      n = doms[d].n;
      s0 = start[d];
      if constexpr (BUF) b = make_bufs<Op>(a, n);
    }
    if constexpr (BUF) tile_buf<Op, BLOCK, PPT, NT>(a, b, n, t - s0);
    else tile<Op, BLOCK, PPT, NT>(a, n, t - s0);
  }
}

__global__ void k_copy(const double* __restrict__ src, double* __restrict__ dst, int64_t n) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x * 2;
  for (int64_t i = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) * 2; i < n;
       i += stride) {
    if (i + 2 <= n && ((reinterpret_cast<uintptr_t>(src + i) | reinterpret_cast<uintptr_t>(dst + i)) & 15) == 0) {
      store2<true>(dst + i, load2<true>(src + i));
    } else {
      dst[i] = src[i];
      if (i + 1 < n) dst[i + 1] = src[i + 1];
    }
  }
}

// Read-only reference: every block sums a grid-stride share of src (16-byte
// non-temporal loads) and writes its partial sum to partial[blockIdx.x].
__global__ __launch_bounds__(256) void k_read(const double* __restrict__ src,
                                             double* __restrict__ partial, int64_t n,
                                             int32_t vec) {
  const int64_t tid = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  const int64_t nth = static_cast<int64_t>(gridDim.x) * 256;
  double s = 0.0;
  if (vec) {
    const int64_t n2 = n / 2;
    for (int64_t i = tid; i < n2; i += nth) {
      const dbl2 v = load2<true>(src + 2 * i);
      s += v.x + v.y;
    }
    if (tid == 0 && (n & 1)) s += src[n - 1];
  } else {
    for (int64_t i = tid; i < n; i += nth) s += load1<true>(src + i);
  }
  __shared__ double red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (static_cast<int>(threadIdx.x) < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// Write-only reference: dst[i] = 1 (16-byte non-temporal stores).
__global__ __launch_bounds__(256) void k_write(double* __restrict__ dst, int64_t n, int32_t vec) {
  const int64_t tid = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  const int64_t nth = static_cast<int64_t>(gridDim.x) * 256;
  if (vec) {
    const int64_t n2 = n / 2;
    const dbl2 one = {1.0, 1.0};
    for (int64_t i = tid; i < n2; i += nth) store2<true>(dst + 2 * i, one);
    if (tid == 0 && (n & 1)) dst[n - 1] = 1.0;
  } else {
    for (int64_t i = tid; i < n; i += nth) store1<true>(dst + i, 1.0);
  }
}

// Christoffel symbols with P neighbouring lanes per grid point: every lane
// loads its point's 24 inputs and evaluates the same body, and stores the
// components q with q mod P == its rank.
template <int P, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_christoffel_lanes(KArgs a, int64_t n) {
  const int64_t gid = static_cast<int64_t>(blockIdx.x) * BLOCK + threadIdx.x;
  const int64_t p = gid / P;
  const int rank = static_cast<int>(gid - p * P);
  if (p >= n) return;
  double x[OpChristoffel::NIN], y[OpChristoffel::NOUT];
#pragma unroll
  for (int c = 0; c < 6; ++c) x[c] = load1<true>(a.in[0] + c * a.ldin[0] + p);
#pragma unroll
  for (int c = 0; c < 18; ++c) x[6 + c] = load1<true>(a.in[1] + c * a.ldin[1] + p);
  OpChristoffel::apply(x, y);
#pragma unroll
  for (int q = 0; q < 18; ++q)
    if (q % P == rank) store1<true>(a.out[0] + q * a.ldout[0] + p, y[q]);
}

template <int P>
static const void* lanes_ptr(int block) {
  switch (block) {
    case 64: return reinterpret_cast<const void*>(&k_christoffel_lanes<P, 64>);
    case 128: return reinterpret_cast<const void*>(&k_christoffel_lanes<P, 128>);
    case 256: return reinterpret_cast<const void*>(&k_christoffel_lanes<P, 256>);
    case 512: return reinterpret_cast<const void*>(&k_christoffel_lanes<P, 512>);
    case 1024: return reinterpret_cast<const void*>(&k_christoffel_lanes<P, 1024>);
    default: return nullptr;
  }
}

static const void* ptr_christoffel_lanes(const Resolved& r) {
  switch (r.lanes) {
    case 2: return lanes_ptr<2>(r.block);
    case 3: return lanes_ptr<3>(r.block);
    case 6: return lanes_ptr<6>(r.block);
    case 9: return lanes_ptr<9>(r.block);
    case 18: return lanes_ptr<18>(r.block);
    default: return nullptr;
  }
}

template <class Op, int BLOCK, int PPT, bool NT, bool BUF>
static const void* batched_ptr() {
  return reinterpret_cast<const void*>(&k_batched<Op, BLOCK, PPT, NT, BUF>);
}

template <class Op, int BLOCK, int PPT>
static const void* batched_ptr_p(const Resolved& r) {
  if (!r.nt) return batched_ptr<Op, BLOCK, PPT, false, false>();
  return r.buf ? batched_ptr<Op, BLOCK, PPT, true, true>()
               : batched_ptr<Op, BLOCK, PPT, true, false>();
}

template <class Op>
static const void* ptr_batched_op(const Resolved& r) {
#define TL_PTR(B) \
  case B:         \
    return r.ppt == 2 ? batched_ptr_p<Op, B, 2>(r) : batched_ptr_p<Op, B, 1>(r);
  switch (r.block) {
    TL_PTR(64)
    TL_PTR(128)
    TL_PTR(256)
    TL_PTR(512)
    TL_PTR(1024)
    default: return nullptr;
  }
#undef TL_PTR
}

static const void* ptr_batched(KernelId k, const Resolved& r) {
  switch (k) {
    case KernelId::ChainBatched: return ptr_batched_op<OpChain>(r);
    case KernelId::ChainBwdBatched: return ptr_batched_op<OpChainBwd>(r);
    default: return nullptr;
  }
}

hipError_t launch_twin(int nin, int nout, const Resolved& r, const KArgs& a, int64_t n,
                       hipStream_t s) {
#define TL_TWIN(I, O) \
  if (nin == I && nout == O) return launch_op<OpTwin<I, O>>(r, a, n, s);
  TL_TWIN_SHAPES(TL_TWIN)
#undef TL_TWIN
  return hipErrorInvalidValue;
}

hipError_t launch_kernel(KernelId k, const Resolved& r, const KArgs& a, int64_t n,
                         hipStream_t s) {
  switch (k) {
    case KernelId::SymInverse: return launch_op<OpSymInverse>(r, a, n, s);
    case KernelId::Christoffel: return launch_op<OpChristoffel>(r, a, n, s);
    case KernelId::CovDeriv: return launch_op<OpCovDeriv>(r, a, n, s);
    case KernelId::Dtg: return launch_op<OpDtg>(r, a, n, s);
    case KernelId::Chain: return launch_op<OpChain>(r, a, n, s);
    case KernelId::ChainBwd: return launch_op<OpChainBwd>(r, a, n, s);
    case KernelId::ChainFwdBwd: return launch_op<OpChainFwdBwd>(r, a, n, s);
    default: return hipErrorInvalidValue;
  }
}

const void* kernel_address(KernelId k, const Resolved& r) {
  switch (k) {
    case KernelId::SymInverse: return ptr_op<OpSymInverse>(r);
    case KernelId::Christoffel:
      return r.lanes > 1 ? ptr_christoffel_lanes(r) : ptr_op<OpChristoffel>(r);
    case KernelId::CovDeriv: return ptr_op<OpCovDeriv>(r);
    case KernelId::Dtg: return ptr_op<OpDtg>(r);
    case KernelId::Chain: return ptr_op<OpChain>(r);
    case KernelId::ChainBwd: return ptr_op<OpChainBwd>(r);
    case KernelId::ChainFwdBwd: return ptr_op<OpChainFwdBwd>(r);
    case KernelId::ChainBatched:
    case KernelId::ChainBwdBatched: return ptr_batched(k, r);
    default: return nullptr;
  }
}

hipError_t launch_batched(KernelId k, const Resolved& r, const BatchDomain* doms, const int64_t* start,
                          const int32_t* tile_dom, int64_t ntiles, int64_t grid, int64_t chunk,
                          hipStream_t s) {
  const void* fn = ptr_batched(k, r);
  if (fn == nullptr) return hipErrorInvalidValue;
  int32_t xcd = r.xcd ? 1 : 0;
  void* args[] = {const_cast<BatchDomain**>(&doms), const_cast<int64_t**>(&start),
                  const_cast<int32_t**>(&tile_dom), &ntiles, &chunk, &xcd};
  hipError_t e = hipLaunchKernel(fn, dim3(static_cast<unsigned>(grid)), dim3(r.block), args, 0, s);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

hipError_t launch_copy(const double* src, double* dst, int64_t n, int64_t grid, hipStream_t s) {
  hipLaunchKernelGGL(k_copy, dim3(static_cast<unsigned>(grid)), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

hipError_t launch_christoffel_lanes(const Resolved& r, const KArgs& a, int64_t n, hipStream_t s) {
  const void* fn = ptr_christoffel_lanes(r);
  if (fn == nullptr) return hipErrorInvalidValue;
  const int64_t grid = (n * r.lanes + r.block - 1) / r.block;
  if (grid > 0x7fffffff) return hipErrorInvalidConfiguration;
  KArgs args = a;
  int64_t npts = n;
  void* kargs[] = {&args, &npts};
  hipError_t e = hipLaunchKernel(fn, dim3(static_cast<unsigned>(grid)), dim3(r.block), kargs, 0, s);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

hipError_t launch_read(const double* src, double* partial, int64_t n, int64_t grid, bool vec,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_read, dim3(static_cast<unsigned>(grid)), dim3(256), 0, s, src, partial, n,
                     vec ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_write(double* dst, int64_t n, int64_t grid, bool vec, hipStream_t s) {
  hipLaunchKernelGGL(k_write, dim3(static_cast<unsigned>(grid)), dim3(256), 0, s, dst, n,
                     vec ? 1 : 0);
  return hipGetLastError();
}

}  // namespace tl
