// Streaming machinery shared by the kernel translation units (device code
// for gfx950, plus the host-side launch templates).
//
// One lane owns PPT consecutive grid points.  It issues every load of its
// points up front -- one coalesced stream per tensor component, 16-byte
// vector loads when PPT is 2 or 4 -- runs the per-point body (tl_device.hpp,
// tl_expr_ops.hpp) in registers and streams the results out.  No LDS and no
// MFMA: every point is independent and the contractions are 3 long, so the
// kernels are bound by HBM bandwidth, and the levers are the bytes in flight
// per CU (PPT, block size, occupancy), the cache policy (non-temporal loads and
// stores), the order in which tiles meet the memory system (XCD order) and
// the instructions spent on addresses (buffer addressing, below).
//
// A body with more outputs than registers comfortably hold (kStream) is
// instead given a loader ld(field, component) and a storer st(field,
// component, value) and interleaves its own loads, math and stores in program
// order, one point per lane; stores are never moved above later loads, so
// only one group of outputs is live at a time.
//
// A tile is BLOCK*PPT consecutive points; a block walks tiles
// logical_block, logical_block + gridDim.x, ... so the same kernel serves a
// grid of one tile per block and a persistent grid.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "tl_internal.hpp"

namespace tl {

typedef double dbl2 __attribute__((ext_vector_type(2)));

template <bool NT>
__device__ inline double load1(const double* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}
template <bool NT>
__device__ inline dbl2 load2(const double* p) {
  const dbl2* q = reinterpret_cast<const dbl2*>(p);
  if constexpr (NT) return __builtin_nontemporal_load(q);
  else return *q;
}
template <bool NT>
__device__ inline void store1(double* p, double v) {
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}
template <bool NT>
__device__ inline void store2(double* p, dbl2 v) {
  dbl2* q = reinterpret_cast<dbl2*>(p);
  if constexpr (NT) __builtin_nontemporal_store(v, q);
  else *q = v;
}

// ---- Buffer addressing.  A wave of a wide body addresses up to 83 component
// streams; with 64-bit pointers every one costs a 64-bit scalar multiply-add
// and the live addresses overflow the scalar registers.  Instead each field
// gets one buffer descriptor (base and extent in bytes) and every access is
// base + lane offset (p * 8, a vector register shared by all components) +
// component offset (c * ld * 8, a 32-bit scalar).  Used when every field's
// extent is below 4 GiB (checked by the host).
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef __amdgpu_buffer_rsrc_t rsrc_t;
constexpr int kRsrcWord3 = 0x00020000;  // raw (unstructured) buffer, gfx9 family
constexpr int kCpolNT = 2;              // the non-temporal cache-policy bit

__device__ inline rsrc_t make_rsrc(const double* base, int64_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(base), 0,
                                           static_cast<int>(static_cast<uint32_t>(bytes)),
                                           kRsrcWord3);
}
template <bool NT>
__device__ inline double bload1(rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(double,
                            __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, NT ? kCpolNT : 0));
}
template <bool NT>
__device__ inline dbl2 bload2(rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(dbl2,
                            __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, NT ? kCpolNT : 0));
}
template <bool NT>
__device__ inline void bstore1(rsrc_t r, uint32_t voff, uint32_t soff, double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, soff,
                                        NT ? kCpolNT : 0);
}
// A store of more than 64 bits reads its data registers after it has issued,
// so an instruction that rewrites them must come two wait states later.  The
// compiler inserts that gap only for a store whose scalar offset operand is
// not a register; with the component offset in a scalar register (as for the
// 8-byte stores) it inserts none, and on gfx950 such a store followed at once
// by a rewrite of its data stored the new value now and then.  So the 16-byte
// store adds the component offset to the lane's vector offset and leaves the
// scalar offset zero: one vector add per store, and a store the compiler pads.
template <bool NT>
__device__ inline void bstore2(rsrc_t r, uint32_t voff, uint32_t soff, dbl2 v) {
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), r, voff + soff, 0,
                                         NT ? kCpolNT : 0);
}

// Offsets of each field's first component in the gathered per-point vector.
template <int NF>
struct Offsets {
  int v[NF + 1];
};
template <class Op>
constexpr Offsets<Op::NF_IN> in_offsets() {
  Offsets<Op::NF_IN> o{};
  o.v[0] = 0;
  for (int f = 0; f < Op::NF_IN; ++f) o.v[f + 1] = o.v[f] + Op::fin[f];
  return o;
}
template <class Op>
constexpr Offsets<Op::NF_OUT> out_offsets() {
  Offsets<Op::NF_OUT> o{};
  o.v[0] = 0;
  for (int f = 0; f < Op::NF_OUT; ++f) o.v[f + 1] = o.v[f] + Op::fout[f];
  return o;
}

// Largest block an Op may run in (Op::kMaxBlock, default 1024): bodies that
// keep many values live would spill to scratch in larger blocks.
template <class Op, class = void>
struct max_block : std::integral_constant<int, 1024> {};
template <class Op>
struct max_block<Op, std::void_t<decltype(Op::kMaxBlock)>>
    : std::integral_constant<int, Op::kMaxBlock> {};

// Streaming bodies (Op::kStream) run one point per lane through ld/st.
template <class Op, class = void>
struct is_stream : std::false_type {};
template <class Op>
struct is_stream<Op, std::void_t<decltype(Op::kStream)>> : std::bool_constant<Op::kStream> {};

// Points per lane a body actually runs with for a requested ppt: streaming
// bodies take one; four only for bodies with at most kMaxStreams4 component
// streams (their four points' values then fit the registers), else two.
constexpr int kMaxStreams4 = 24;
template <class Op>
constexpr int op_ppt(int ppt) {
  if constexpr (is_stream<Op>::value) return 1;
  else return ppt == 4 && Op::NIN + Op::NOUT > kMaxStreams4 ? 2 : ppt;
}

template <class Op, bool NT>
__device__ inline void point_stream(const KArgs& a, int64_t p) {
  Op::stream([&](int f, int c) { return load1<NT>(a.in[f] + c * a.ldin[f] + p); },
             [&](int f, int c, double v) { store1<NT>(a.out[f] + c * a.ldout[f] + p, v); });
}

// Points p .. p+PPT-1 of one tile, all in range.
template <class Op, int PPT, bool NT>
__device__ inline void points_full(const KArgs& a, int64_t p, int64_t hs = 0) {
  constexpr auto io = in_offsets<Op>();
  constexpr auto oo = out_offsets<Op>();
  if constexpr (PPT == 1) {
    double x[Op::NIN], y[Op::NOUT];
#pragma unroll
    for (int f = 0; f < Op::NF_IN; ++f)
#pragma unroll
      for (int c = 0; c < Op::fin[f]; ++c) x[io.v[f] + c] = load1<NT>(a.in[f] + c * a.ldin[f] + p);
    Op::apply(x, y);
#pragma unroll
    for (int f = 0; f < Op::NF_OUT; ++f) {
      if (a.out[f] == nullptr) continue;
#pragma unroll
      for (int c = 0; c < Op::fout[f]; ++c) store1<NT>(a.out[f] + c * a.ldout[f] + p, y[oo.v[f] + c]);
    }
  } else {
    static_assert(PPT == 2 || PPT == 4, "PPT is 1, 2 or 4");
    constexpr int H = PPT / 2;  // point pairs, hs points apart: 16-byte accesses per component
    dbl2 x2[H][Op::NIN];
#pragma unroll
    for (int f = 0; f < Op::NF_IN; ++f)
#pragma unroll
      for (int c = 0; c < Op::fin[f]; ++c)
#pragma unroll
        for (int h = 0; h < H; ++h)
          x2[h][io.v[f] + c] = load2<NT>(a.in[f] + c * a.ldin[f] + p + h * hs);
    double x[Op::NIN], y[PPT][Op::NOUT];
#pragma unroll
    for (int h = 0; h < H; ++h) {
#pragma unroll
      for (int q = 0; q < Op::NIN; ++q) x[q] = x2[h][q].x;
      Op::apply(x, y[2 * h]);
#pragma unroll
      for (int q = 0; q < Op::NIN; ++q) x[q] = x2[h][q].y;
      Op::apply(x, y[2 * h + 1]);
    }
#pragma unroll
    for (int f = 0; f < Op::NF_OUT; ++f) {
      if (a.out[f] == nullptr) continue;
#pragma unroll
      for (int c = 0; c < Op::fout[f]; ++c)
#pragma unroll
        for (int h = 0; h < H; ++h) {
          dbl2 v;
          v.x = y[2 * h][oo.v[f] + c];
          v.y = y[2 * h + 1][oo.v[f] + c];
          store2<NT>(a.out[f] + c * a.ldout[f] + p + h * hs, v);
        }
    }
  }
}

// Points p .. min(p+PPT, n)-1, scalar accesses (the ragged tail).
template <class Op, int PPT>
__device__ inline void points_tail(const KArgs& a, int64_t p, int64_t n) {
  constexpr auto io = in_offsets<Op>();
  constexpr auto oo = out_offsets<Op>();
  for (int k = 0; k < PPT; ++k) {
    const int64_t q = p + k;
    if (q >= n) break;
    double x[Op::NIN], y[Op::NOUT];
#pragma unroll
    for (int f = 0; f < Op::NF_IN; ++f)
#pragma unroll
      for (int c = 0; c < Op::fin[f]; ++c) x[io.v[f] + c] = a.in[f][c * a.ldin[f] + q];
    Op::apply(x, y);
#pragma unroll
    for (int f = 0; f < Op::NF_OUT; ++f) {
      if (a.out[f] == nullptr) continue;
#pragma unroll
      for (int c = 0; c < Op::fout[f]; ++c) a.out[f][c * a.ldout[f] + q] = y[oo.v[f] + c];
    }
  }
}

// One descriptor and one component stride (bytes) per field.
template <class Op>
struct Bufs {
  rsrc_t in[Op::NF_IN], out[Op::NF_OUT];
  uint32_t ldin8[Op::NF_IN], ldout8[Op::NF_OUT];
};

template <class Op>
__device__ inline Bufs<Op> make_bufs(const KArgs& a, int64_t n) {
  Bufs<Op> b;
#pragma unroll
  for (int f = 0; f < Op::NF_IN; ++f) {
    b.in[f] = make_rsrc(a.in[f], ((Op::fin[f] - 1) * a.ldin[f] + n) * 8);
    b.ldin8[f] = static_cast<uint32_t>(a.ldin[f] * 8);
  }
#pragma unroll
  for (int f = 0; f < Op::NF_OUT; ++f) {
    b.out[f] = make_rsrc(a.out[f], ((Op::fout[f] - 1) * a.ldout[f] + n) * 8);
    b.ldout8[f] = static_cast<uint32_t>(a.ldout[f] * 8);
  }
  return b;
}

template <class Op, bool NT>
__device__ inline void point_stream_buf(const Bufs<Op>& b, uint32_t p8) {
  Op::stream([&](int f, int c) { return bload1<NT>(b.in[f], p8, c * b.ldin8[f]); },
             [&](int f, int c, double v) { bstore1<NT>(b.out[f], p8, c * b.ldout8[f], v); });
}

template <class Op, int PPT, bool NT>
__device__ inline void points_full_buf(const KArgs& a, const Bufs<Op>& b, uint32_t p8,
                                       uint32_t hs8 = 0) {
  constexpr auto io = in_offsets<Op>();
  constexpr auto oo = out_offsets<Op>();
  if constexpr (PPT == 1) {
    double x[Op::NIN], y[Op::NOUT];
#pragma unroll
    for (int f = 0; f < Op::NF_IN; ++f)
#pragma unroll
      for (int c = 0; c < Op::fin[f]; ++c) x[io.v[f] + c] = bload1<NT>(b.in[f], p8, c * b.ldin8[f]);
    Op::apply(x, y);
#pragma unroll
    for (int f = 0; f < Op::NF_OUT; ++f) {
      if (a.out[f] == nullptr) continue;
#pragma unroll
      for (int c = 0; c < Op::fout[f]; ++c)
        bstore1<NT>(b.out[f], p8, c * b.ldout8[f], y[oo.v[f] + c]);
    }
  } else {
    static_assert(PPT == 2 || PPT == 4, "PPT is 1, 2 or 4");
    constexpr int H = PPT / 2;  // point pairs, hs points apart: 16-byte accesses per component
    dbl2 x2[H][Op::NIN];
#pragma unroll
    for (int f = 0; f < Op::NF_IN; ++f)
#pragma unroll
      for (int c = 0; c < Op::fin[f]; ++c)
#pragma unroll
        for (int h = 0; h < H; ++h)
          x2[h][io.v[f] + c] = bload2<NT>(b.in[f], p8 + h * hs8, c * b.ldin8[f]);
    double x[Op::NIN], y[PPT][Op::NOUT];
#pragma unroll
    for (int h = 0; h < H; ++h) {
#pragma unroll
      for (int q = 0; q < Op::NIN; ++q) x[q] = x2[h][q].x;
      Op::apply(x, y[2 * h]);
#pragma unroll
      for (int q = 0; q < Op::NIN; ++q) x[q] = x2[h][q].y;
      Op::apply(x, y[2 * h + 1]);
    }
#pragma unroll
    for (int f = 0; f < Op::NF_OUT; ++f) {
      if (a.out[f] == nullptr) continue;
#pragma unroll
      for (int c = 0; c < Op::fout[f]; ++c)
#pragma unroll
        for (int h = 0; h < H; ++h) {
          dbl2 v;
          v.x = y[2 * h][oo.v[f] + c];
          v.y = y[2 * h + 1][oo.v[f] + c];
          bstore2<NT>(b.out[f], p8 + h * hs8, c * b.ldout8[f], v);
        }
    }
  }
}

// A tile is BLOCK*PPT consecutive points.  With PPT of 1 or 2 a lane owns PPT
// consecutive points of it; with PPT = 4 a lane owns two pairs of points, one
// in each half of the tile (2*BLOCK points apart), so every 16-byte access of a
// wave still covers a contiguous kilobyte.
template <class Op, int BLOCK, int PPT, bool NT>
__device__ inline void tile_buf(const KArgs& a, const Bufs<Op>& b, int64_t n, int64_t t) {
  if constexpr (is_stream<Op>::value) {
    static_assert(PPT == 1, "streaming bodies take one point per lane");
    const int64_t p = t * BLOCK + threadIdx.x;
    if (p < n) point_stream_buf<Op, NT>(b, static_cast<uint32_t>(p * 8));
  } else if constexpr (PPT == 4) {
    const int64_t p = t * BLOCK * 4 + 2 * threadIdx.x;
    const int64_t q = p + 2 * BLOCK;
    if (q + 2 <= n) {
      points_full_buf<Op, 4, NT>(a, b, static_cast<uint32_t>(p * 8), 16u * BLOCK);
    } else {
      if (p + 2 <= n) points_full_buf<Op, 2, NT>(a, b, static_cast<uint32_t>(p * 8));
      else if (p < n) points_tail<Op, 2>(a, p, n);
      if (q < n) points_tail<Op, 2>(a, q, n);
    }
  } else {
    const int64_t p = (t * BLOCK + threadIdx.x) * PPT;
    if (p + PPT <= n) points_full_buf<Op, PPT, NT>(a, b, static_cast<uint32_t>(p * 8));
    else if (p < n) points_tail<Op, PPT>(a, p, n);
  }
}

template <class Op, int BLOCK, int PPT, bool NT>
__device__ inline void tile(const KArgs& a, int64_t n, int64_t t) {
  if constexpr (is_stream<Op>::value) {
    static_assert(PPT == 1, "streaming bodies take one point per lane");
    const int64_t p = t * BLOCK + threadIdx.x;
    if (p < n) point_stream<Op, NT>(a, p);
  } else if constexpr (PPT == 4) {
    const int64_t p = t * BLOCK * 4 + 2 * threadIdx.x;
    const int64_t q = p + 2 * BLOCK;
    if (q + 2 <= n) {
      points_full<Op, 4, NT>(a, p, 2 * BLOCK);
    } else {
      if (p + 2 <= n) points_full<Op, 2, NT>(a, p);
      else if (p < n) points_tail<Op, 2>(a, p, n);
      if (q < n) points_tail<Op, 2>(a, q, n);
    }
  } else {
    const int64_t p = (t * BLOCK + threadIdx.x) * PPT;
    if (p + PPT <= n) points_full<Op, PPT, NT>(a, p);
    else if (p < n) points_tail<Op, PPT>(a, p, n);
  }
}

// Logical block index.  Workgroups are dispatched to the 8 XCDs round-robin
// (block b runs on XCD b % 8); with `xcd` set (and gridDim.x a multiple of
// 8) the blocks of one XCD take a contiguous run of tiles instead of every
// 8th tile, so each XCD streams through its own contiguous address ranges.
__device__ inline int64_t logical_block(int32_t xcd) {
  const int64_t b = blockIdx.x;
  if (!xcd) return b;
  const int64_t per = gridDim.x >> 3;
  return (b & 7) * per + (b >> 3);
}

// BUF: buffer addressing (every field's extent below 4 GiB); otherwise 64-bit
// pointers.
template <class Op, int BLOCK, int PPT, bool NT, bool BUF>
__global__ __launch_bounds__(BLOCK) void k_points(KArgs a, int64_t n, int64_t ntiles, int32_t xcd) {
  if constexpr (BUF) {
    const Bufs<Op> b = make_bufs<Op>(a, n);
    for (int64_t t = logical_block(xcd); t < ntiles; t += gridDim.x)
      tile_buf<Op, BLOCK, PPT, NT>(a, b, n, t);
  } else {
    for (int64_t t = logical_block(xcd); t < ntiles; t += gridDim.x)
      tile<Op, BLOCK, PPT, NT>(a, n, t);
  }
}


template <class Op, int BLOCK, int PPT, bool NT, bool BUF>
static const void* kernel_ptr() {
  return reinterpret_cast<const void*>(&k_points<Op, BLOCK, PPT, NT, BUF>);
}

template <class Op, int BLOCK, int PPT, bool NT, bool BUF>
static hipError_t launch_one(const KArgs& a, int64_t n, int64_t ntiles, int64_t grid, int32_t xcd,
                             hipStream_t s) {
  hipLaunchKernelGGL((k_points<Op, BLOCK, PPT, NT, BUF>), dim3(static_cast<unsigned>(grid)),
                     dim3(BLOCK), 0, s, a, n, ntiles, xcd);
  return hipGetLastError();
}

// Buffer addressing is instantiated with the non-temporal hint only (the
// default); a request without it takes the pointer path.
template <class Op, int BLOCK, int PPT>
static hipError_t launch_p(const Resolved& r, const KArgs& a, int64_t n, int64_t ntiles,
                           int64_t grid, int32_t x, hipStream_t s) {
  if (!r.nt) return launch_one<Op, BLOCK, PPT, false, false>(a, n, ntiles, grid, x, s);
  return r.buf ? launch_one<Op, BLOCK, PPT, true, true>(a, n, ntiles, grid, x, s)
               : launch_one<Op, BLOCK, PPT, true, false>(a, n, ntiles, grid, x, s);
}

template <class Op, int BLOCK>
static hipError_t launch_b(const Resolved& r, const KArgs& a, int64_t n, int64_t ntiles,
                           int64_t grid, hipStream_t s) {
  const int32_t x = r.xcd ? 1 : 0;
  if constexpr (is_stream<Op>::value) {
    return launch_p<Op, BLOCK, 1>(r, a, n, ntiles, grid, x, s);
  } else {
    const int ppt = op_ppt<Op>(r.ppt);
    if constexpr (Op::NIN + Op::NOUT <= kMaxStreams4)
      if (ppt == 4) return launch_p<Op, BLOCK, 4>(r, a, n, ntiles, grid, x, s);
    if (ppt == 2) return launch_p<Op, BLOCK, 2>(r, a, n, ntiles, grid, x, s);
    return launch_p<Op, BLOCK, 1>(r, a, n, ntiles, grid, x, s);
  }
}

template <class Op>
static Resolved clamp_block(const Resolved& r0) {
  Resolved r = r0;
  if (r.block > max_block<Op>::value) r.block = max_block<Op>::value;
  return r;
}

template <class Op>
static hipError_t launch_op(const Resolved& r0, const KArgs& a, int64_t n, hipStream_t s) {
  const Resolved r = clamp_block<Op>(r0);
  const int64_t per = static_cast<int64_t>(r.block) * op_ppt<Op>(r.ppt);
  const int64_t ntiles = (n + per - 1) / per;
  const int64_t grid = grid_size(r, ntiles);
  constexpr int cap = max_block<Op>::value;
  switch (r.block) {
    case 64: return launch_b<Op, 64>(r, a, n, ntiles, grid, s);
    case 128: return launch_b<Op, 128>(r, a, n, ntiles, grid, s);
    case 256: return launch_b<Op, 256>(r, a, n, ntiles, grid, s);
    case 512:
      if constexpr (cap >= 512) return launch_b<Op, 512>(r, a, n, ntiles, grid, s);
      return hipErrorInvalidValue;
    case 1024:
      if constexpr (cap >= 1024) return launch_b<Op, 1024>(r, a, n, ntiles, grid, s);
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

template <class Op, int BLOCK, int PPT>
static const void* ptr_p(const Resolved& r) {
  if (!r.nt) return kernel_ptr<Op, BLOCK, PPT, false, false>();
  return r.buf ? kernel_ptr<Op, BLOCK, PPT, true, true>() : kernel_ptr<Op, BLOCK, PPT, true, false>();
}

template <class Op, int BLOCK>
static const void* ptr_b(const Resolved& r) {
  if constexpr (is_stream<Op>::value) {
    return ptr_p<Op, BLOCK, 1>(r);
  } else {
    const int ppt = op_ppt<Op>(r.ppt);
    if constexpr (Op::NIN + Op::NOUT <= kMaxStreams4)
      if (ppt == 4) return ptr_p<Op, BLOCK, 4>(r);
    return ppt == 2 ? ptr_p<Op, BLOCK, 2>(r) : ptr_p<Op, BLOCK, 1>(r);
  }
}

template <class Op>
static const void* ptr_op(const Resolved& r0) {
  const Resolved r = clamp_block<Op>(r0);
  constexpr int cap = max_block<Op>::value;
#define TL_PTR(B)                                 \
  case B:                                         \
    if constexpr (cap >= B) return ptr_b<Op, B>(r); \
    return nullptr;
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

}  // namespace tl
