// The batched forward chain with its tables in a fixed device array, for
// callers that cannot allocate device memory (tl_batch_run_noalloc).
//
// A batch plan keeps three tables in device memory it allocates: the domain
// descriptors, the first tile of every domain, and the tile -> domain map.
// Here they live in `scratch`, one file-scope array per device, and are
// written by small kernels that receive the descriptors as kernel arguments
// (so the call makes no memory copy of its own and allocates nothing); the
// batched kernel of the plans then reads them from there.
#include <hip/hip_runtime.h>

#include <cstddef>
#include <mutex>

#include "tl_internal.hpp"

namespace tl {
namespace {

// Layout of the array: [domains][tile starts][tile -> domain map].
constexpr int64_t kDomBytes = static_cast<int64_t>(sizeof(BatchDomain)) * TL_NOALLOC_MAX_DOMAINS;
constexpr int64_t kStartOff = kDomBytes;
constexpr int64_t kStartBytes = (8 * (TL_NOALLOC_MAX_DOMAINS + 1) + 255) / 256 * 256;
constexpr int64_t kTileOff = kStartOff + kStartBytes;
constexpr int64_t kScratchBytes = kTileOff + 4 * static_cast<int64_t>(TL_NOALLOC_MAX_TILES);
static_assert(kDomBytes % 256 == 0, "tile starts must stay 256-byte aligned");

// Each device holds its own copy until the process ends.  Host code never
// uses this name as an address: it asks the runtime for the device's copy
// (scratch_base) and passes that pointer on.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_base[kMaxDevices] = {};

// Address of the current device's copy of `scratch`, looked up once per
// device with that device current.
hipError_t scratch_base(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_base[dev] == nullptr) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (p == nullptr) return hipErrorInvalidSymbol;
    g_base[dev] = p;
  }
  *out = g_base[dev];
  return hipSuccess;
}

// The 64-bit words of a BatchDomain that a forward-chain domain sets (its six
// input fields, one output field and n); every other word is zero.
constexpr int kDomWords = static_cast<int>(sizeof(BatchDomain) / 8);
constexpr int kSetWords = 15;
constexpr int word_of(int k) {  // word of the BatchDomain that packed word k fills
  return k < 6 ? k                                  // args.in[0..5]
       : k < 12 ? kMaxFields + (k - 6)               // args.ldin[0..5]
       : k == 12 ? 2 * kMaxFields                    // args.out[0]
       : k == 13 ? 3 * kMaxFields                    // args.ldout[0]
       : 4 * kMaxFields;                             // n
}
static_assert(word_of(14) * 8 == offsetof(BatchDomain, n), "BatchDomain layout");
static_assert(kDomWords <= 64, "one wave writes a descriptor");

// Packed descriptors of up to kFillCap consecutive domains, passed by value as
// a kernel argument; with the kernel's three pointers it stays within 4 KB,
// the kernel-argument size every HIP runtime accepts.
constexpr int kFillCap = 31;
struct FillChunk {
  int32_t d0, nd;                   // domains d0 .. d0 + nd - 1
  int64_t start[kFillCap + 1];      // their first tiles, then the tile after the last
  int64_t w[kFillCap][kSetWords];   // word k of domain i: see word_of(k)
};
static_assert(sizeof(FillChunk) + 3 * sizeof(void*) <= 4096, "kernel argument too large");

// Block 0 writes the chunk's descriptors (lane l of the first wave writes word
// l of each, so a descriptor is one store) and tile starts; every lane of the
// grid then writes the domain of one tile of the chunk: the last domain whose
// first tile is not after it (domains without tiles are passed over because
// the next one starts at the same tile).  The argument words a block uses are
// first copied to LDS by all its lanes at once, so the argument (which the
// runtime may keep in host memory) is read in one round trip rather than one
// per dependent load.
__global__ __launch_bounds__(256) void k_fill_tables(FillChunk c, BatchDomain* __restrict__ doms,
                                                     int64_t* __restrict__ start,
                                                     int32_t* __restrict__ tile_dom) {
  __shared__ int64_t s_start[kFillCap + 1];
  __shared__ int64_t s_w[kFillCap * kSetWords];
  const int l = threadIdx.x;
  const int nd = c.nd;
  if (l <= nd) s_start[l] = c.start[l];
  if (blockIdx.x == 0) {
    const int64_t* w = &c.w[0][0];
    for (int q = l; q < nd * kSetWords; q += 256) s_w[q] = w[q];
  }
  __syncthreads();
  if (blockIdx.x == 0) {
    int k = -1;  // the packed word this lane writes, if any
#pragma unroll
    for (int q = 0; q < kSetWords; ++q)
      if (word_of(q) == l) k = q;
    if (l < kDomWords) {
      int64_t* out = reinterpret_cast<int64_t*>(doms + c.d0);
      for (int i = 0; i < nd; ++i) out[i * kDomWords + l] = k >= 0 ? s_w[i * kSetWords + k] : 0;
    }
    if (l <= nd) start[c.d0 + l] = s_start[l];
  }
  const int64_t t = s_start[0] + static_cast<int64_t>(blockIdx.x) * 256 + l;
  if (t < s_start[nd]) {
    int32_t i = 0;
    for (int j = 1; j < nd; ++j) i += s_start[j] <= t ? 1 : 0;
    tile_dom[t] = c.d0 + i;
  }
}

}  // namespace

hipError_t launch_batched_noalloc(const Resolved& r, const BatchDomain* doms,
                                  const int64_t* start, int32_t ndom, int64_t ntiles,
                                  int64_t grid, int64_t chunk, hipStream_t s) {
  if (ndom < 1 || ndom > TL_NOALLOC_MAX_DOMAINS || ntiles < 0 || ntiles > TL_NOALLOC_MAX_TILES ||
      start[ndom] != ntiles)
    return hipErrorInvalidValue;
  void* base = nullptr;
  hipError_t e = scratch_base(&base);
  if (e != hipSuccess) return e;
  unsigned char* b = static_cast<unsigned char*>(base);
  BatchDomain* d_doms = reinterpret_cast<BatchDomain*>(b);
  int64_t* d_start = reinterpret_cast<int64_t*>(b + kStartOff);
  int32_t* d_tile_dom = reinterpret_cast<int32_t*>(b + kTileOff);
  for (int32_t d0 = 0; d0 < ndom; d0 += kFillCap) {
    FillChunk c = {};
    c.d0 = d0;
    c.nd = ndom - d0 < kFillCap ? ndom - d0 : kFillCap;
    for (int i = 0; i < c.nd; ++i) {
      const BatchDomain& x = doms[d0 + i];
      c.start[i] = start[d0 + i];
      for (int f = 0; f < 6; ++f) {
        c.w[i][f] = reinterpret_cast<intptr_t>(x.args.in[f]);
        c.w[i][6 + f] = x.args.ldin[f];
      }
      c.w[i][12] = reinterpret_cast<intptr_t>(x.args.out[0]);
      c.w[i][13] = x.args.ldout[0];
      c.w[i][14] = x.n;
    }
    c.start[c.nd] = start[d0 + c.nd];
    const int64_t tiles = c.start[c.nd] - c.start[0];
    const int64_t blocks = tiles > 0 ? (tiles + 255) / 256 : 1;
    hipLaunchKernelGGL(k_fill_tables, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, c,
                       d_doms, d_start, d_tile_dom);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (ntiles == 0) return hipSuccess;
  return launch_batched(KernelId::ChainBatched, r, d_doms, d_start, d_tile_dom, ntiles, grid,
                        chunk, s);
}

}  // namespace tl
