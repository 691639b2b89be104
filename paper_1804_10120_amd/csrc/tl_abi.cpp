// C ABI of libtl.so: argument validation, tuning resolution, launches, batch
// plans (device descriptor table + HIP graph) and error reporting.  The
// argument checks are the library's counterpart of the paper's extent and
// index checks on assignment (Sec. 2.4): every field must cover the n points
// of the call, and an output may not overlap anything else.
#include "../../include/tl.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "tl_internal.hpp"

namespace {

thread_local std::string g_last_error;

tl_status fail(tl_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

tl_status hip_fail(hipError_t e, const char* what) {
  return fail(TL_ERR_HIP, "%s: %s (%d)", what, hipGetErrorString(e), static_cast<int>(e));
}

// A field as validated: byte range [lo, hi) from its first to its last
// element, and the layout inside it (ncomp components of comp bytes, stride
// bytes apart) for the exact check.
struct Span {
  const char* name;
  uintptr_t lo, hi;
  bool output;
  uintptr_t comp, stride;
  int ncomp;
};

struct Checker {
  int64_t n;
  std::vector<Span> spans;
  bool vec_ok = true;  // every field 16-byte aligned with even ld (for ppt = 2)
  bool buf_ok = true;  // every field spans less than 4 GiB (32-bit buffer offsets)
  tl_status st = TL_OK;

  explicit Checker(int64_t n_) : n(n_) {}

  void field(const char* name, const void* ptr, int64_t ld, int ncomp, bool output,
             bool optional = false) {
    if (st != TL_OK) return;
    if (ptr == nullptr) {
      if (optional) return;
      st = fail(TL_ERR_NULL, "%s is NULL", name);
      return;
    }
    if (ncomp == 1) ld = n;
    if (ld < n) {
      st = fail(TL_ERR_SIZE, "%s: ld=%lld < n=%lld", name, (long long)ld, (long long)n);
      return;
    }
    if (ld > (INT64_MAX / 8 - n) / ncomp) {
      st = fail(TL_ERR_SIZE, "%s: ld=%lld too large", name, (long long)ld);
      return;
    }
    const uintptr_t a = reinterpret_cast<uintptr_t>(ptr);
    if (a % 8 != 0) {
      st = fail(TL_ERR_ALIGN, "%s is not 8-byte aligned", name);
      return;
    }
    if (a % 16 != 0 || (ncomp > 1 && ld % 2 != 0)) vec_ok = false;
    const uintptr_t bytes = static_cast<uintptr_t>((ncomp - 1) * ld + n) * 8u;
    if (bytes > 0xFFFFFFFFull) buf_ok = false;
    spans.push_back({name, a, a + bytes, output, static_cast<uintptr_t>(n) * 8u,
                     static_cast<uintptr_t>(ld) * 8u, ncomp});
  }

  tl_status overlaps() {
    if (st != TL_OK) return st;
    const char* x = nullptr;
    const char* y = nullptr;
    if (overlapping(spans, &x, &y)) return st = fail(TL_ERR_ALIAS, "%s overlaps %s", x, y);
    return st;
  }

  // Whether an output shares a byte with another field.  The whole spans are
  // compared first; only if two of them meet are the individual components
  // compared, so fields interleaved in one buffer (e.g. point ranges of one
  // large field) are accepted when no element is shared.
  static bool overlapping(std::vector<Span>& v, const char** x, const char** y) {
    const Span* a = nullptr;
    const Span* b = nullptr;
    if (!find_overlap(v, &a, &b)) return false;
    std::vector<Span> parts;
    for (const Span& s : v)
      for (int c = 0; c < s.ncomp; ++c) {
        const uintptr_t lo = s.lo + static_cast<uintptr_t>(c) * s.stride;
        parts.push_back({s.name, lo, lo + s.comp, s.output, s.comp, 0, 1});
      }
    if (!find_overlap(parts, &a, &b)) return false;
    *x = a->name;
    *y = b->name;
    return true;
  }

  // Finds a pair of overlapping spans of which at least one is an output
  // (inputs may overlap each other).  Sort by start, then sweep: a span that
  // starts before the furthest end of the outputs seen so far overlaps an
  // output; an output that starts before the furthest end of any span seen so
  // far overlaps that span.  O(S log S).
  static bool find_overlap(std::vector<Span>& v, const Span** x, const Span** y) {
    std::sort(v.begin(), v.end(), [](const Span& p, const Span& q) { return p.lo < q.lo; });
    const Span* far_out = nullptr;  // output with the largest end so far
    const Span* far_any = nullptr;  // span with the largest end so far
    for (const Span& s : v) {
      if (s.hi == s.lo) continue;
      if (far_out && s.lo < far_out->hi) {
        *x = far_out;
        *y = &s;
        return true;
      }
      if (s.output && far_any && s.lo < far_any->hi) {
        *x = far_any;
        *y = &s;
        return true;
      }
      if (!far_any || s.hi > far_any->hi) far_any = &s;
      if (s.output && (!far_out || s.hi > far_out->hi)) far_out = &s;
    }
    return false;
  }
};

// Compute units of the current device (cached per device; calls may come
// from several threads).
int num_cus() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  static std::atomic<int> cache[64];
  if (dev >= 0 && dev < 64) {
    const int c = cache[dev].load(std::memory_order_relaxed);
    if (c > 0) return c;
  }
  int cu = 0;
  if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cu <= 0)
    cu = 256;
  if (dev >= 0 && dev < 64) cache[dev].store(cu, std::memory_order_relaxed);
  return cu;
}

// Default launch shapes, measured on MI355X with the library's autotuner.
// Every kernel streams, so one rule serves nearly all of them: non-temporal
// loads and stores always; for large grids one point per lane in blocks of 256,
// with XCD-contiguous tiles when every XCD's share of each component is 1 or
// 2 MiB (2^20 or 2^21 points), in plain order otherwise (measured for every
// step kernel at 1 to 8 Mi points: the XCD order is 6-33 % faster at those two
// sizes, and at the other sizes tried, powers of two included, up to 16 %
// slower for all but the kernels with the fewest streams); below 2^20
// points (where the whole grid is in
// flight at once and the XCD order buys nothing) two points per lane in
// blocks of 512, except the fused forward, which keeps one point per lane in
// blocks of 256 (62 registers against 166 at two points); below 2^16 points
// (a few memory round trips in all) one point per lane in blocks of 64, to
// spread the grid over as many compute units as possible.  The batched
// kernel: one block of 128 per tile in plain order (its subgrids are already
// contiguous runs of tiles; a persistent grid measured 20% slower than
// letting the dispatcher balance the uneven subgrids).
tl::Resolved defaults(tl::KernelId k, int64_t n) {
  tl::Resolved r;
  r.nt = true;
  r.grid_mult = 0;
  if (k == tl::KernelId::ChainBatched || k == tl::KernelId::ChainBwdBatched) {
    r.block = 128;
    r.ppt = 1;
    r.xcd = false;
  } else if (n >= (int64_t(1) << 20)) {
    r.block = 256;
    r.ppt = 1;
    r.xcd = n == (int64_t(1) << 20) || n == (int64_t(1) << 21);
  } else if (n < (int64_t(1) << 16)) {
    r.block = 64;
    r.ppt = 1;
    r.xcd = false;
  } else if (k == tl::KernelId::Chain || k == tl::KernelId::Generic) {
    r.block = 256;
    r.ppt = 1;
    r.xcd = false;
  } else {
    r.block = 512;
    r.ppt = 2;
    r.xcd = false;
  }
  return r;
}

tl_status resolve(tl::KernelId k, const tl_tune* t, bool vec_ok, bool buf_ok, int64_t n,
                  tl::Resolved* out) {
  tl::Resolved r = defaults(k, n);
  if (t != nullptr) {
    const int l = t->lanes;
    if (l != 0 && l != 1 && l != 2 && l != 3 && l != 6 && l != 9 && l != 18)
      return fail(TL_ERR_INVALID, "tune.lanes=%d not in {0,1,2,3,6,9,18}", l);
    if (l > 1 && k != tl::KernelId::Christoffel)
      return fail(TL_ERR_INVALID, "tune.lanes=%d: only tl_christoffel spreads a point over lanes", l);
    r.lanes = l > 1 ? l : 1;
    if (t->block != 0) {
      if (t->block != 64 && t->block != 128 && t->block != 256 && t->block != 512 &&
          t->block != 1024)
        return fail(TL_ERR_INVALID, "tune.block=%d not in {64,128,256,512,1024}", t->block);
      r.block = t->block;
    }
    if (t->ppt != 0) {
      if (t->ppt != 1 && t->ppt != 2 && t->ppt != 4)
        return fail(TL_ERR_INVALID, "tune.ppt=%d not in {1,2,4}", t->ppt);
      r.ppt = t->ppt;
    }
    if (t->flags & ~(TL_TUNE_NT | TL_TUNE_XCD | TL_TUNE_PTR64))
      return fail(TL_ERR_INVALID, "tune.flags=%d has unknown bits", t->flags);
    r.nt = (t->flags & TL_TUNE_NT) != 0;
    r.xcd = (t->flags & TL_TUNE_XCD) != 0;
    if (t->flags & TL_TUNE_PTR64) buf_ok = false;
    if (t->grid_mult < 0 || t->grid_mult > 1024)
      return fail(TL_ERR_INVALID, "tune.grid_mult=%d not in [0,1024]", t->grid_mult);
    r.grid_mult = t->grid_mult;
  }
  // Four points per lane only where the body's values fit the registers
  // (the inverse and d_t g from nabla beta; a generic body decides on the
  // device), else two.
  if (r.ppt == 4 && k != tl::KernelId::SymInverse && k != tl::KernelId::Dtg &&
      k != tl::KernelId::Generic)
    r.ppt = 2;
  if (!vec_ok) r.ppt = 1;
  r.buf = buf_ok;
  r.num_cu = num_cus();
  *out = r;
  return TL_OK;
}

tl_status run(tl::KernelId k, const Checker& c, const tl_tune* tune, const tl::KArgs& a,
              void* stream) {
  tl::Resolved r;
  tl_status s = resolve(k, tune, c.vec_ok, c.buf_ok, c.n, &r);
  if (s != TL_OK) return s;
  hipError_t e = r.lanes > 1
                     ? tl::launch_christoffel_lanes(r, a, c.n, static_cast<hipStream_t>(stream))
                     : tl::launch_kernel(k, r, a, c.n, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  return TL_OK;
}

tl::KArgs zero_args() {
  tl::KArgs a;
  std::memset(&a, 0, sizeof(a));
  return a;
}

void set_in(tl::KArgs& a, int f, tl_cfield x) {
  a.in[f] = x.ptr;
  a.ldin[f] = x.ld;
}
void set_out(tl::KArgs& a, int f, tl_field x) {
  a.out[f] = x.ptr;
  a.ldout[f] = x.ld;
}

}  // namespace

struct tl_batch_plan {
  int device = 0;
  tl::KernelId kid = tl::KernelId::ChainBatched;
  tl::Resolved r;
  int32_t ndom = 0;
  int64_t points = 0, ntiles = 0, grid = 0, chunk = 1;
  tl::BatchDomain* d_doms = nullptr;
  int64_t* d_start = nullptr;
  int32_t* d_tile_dom = nullptr;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace tl {

tl_status run_generated(const char* name, int64_t n, const tl_cfield* in, int32_t nin,
                        const int32_t* in_ncomp, int32_t nin_expected, const tl_field* out,
                        int32_t nout, const int32_t* out_ncomp, int32_t nout_expected,
                        void* stream, const tl_tune* tune, LaunchFn launch) {
  if (nin != nin_expected || nout != nout_expected)
    return fail(TL_ERR_INVALID, "%s takes %d inputs and %d outputs, got %d and %d", name,
                nin_expected, nout_expected, nin, nout);
  if (nin > kMaxFields || nout > kMaxFields)
    return fail(TL_ERR_INVALID, "%s: more than %d fields", name, kMaxFields);
  if (n < 0) return fail(TL_ERR_SIZE, "n=%lld < 0", (long long)n);
  if (n == 0) return TL_OK;
  if (in == nullptr || out == nullptr) return fail(TL_ERR_NULL, "in or out is NULL");
  static const char* const in_names[kMaxFields] = {"in[0]", "in[1]", "in[2]", "in[3]",
                                                   "in[4]", "in[5]", "in[6]", "in[7]"};
  static const char* const out_names[kMaxFields] = {"out[0]", "out[1]", "out[2]", "out[3]",
                                                    "out[4]", "out[5]", "out[6]", "out[7]"};
  Checker c(n);
  for (int f = 0; f < nin; ++f) c.field(in_names[f], in[f].ptr, in[f].ld, in_ncomp[f], false);
  for (int f = 0; f < nout; ++f)
    c.field(out_names[f], out[f].ptr, out[f].ld, out_ncomp[f], true);
  if (c.overlaps() != TL_OK) return c.st;
  KArgs a = zero_args();
  for (int f = 0; f < nin; ++f) set_in(a, f, in[f]);
  for (int f = 0; f < nout; ++f) set_out(a, f, out[f]);
  Resolved r;
  tl_status s = resolve(KernelId::Generic, tune, c.vec_ok, c.buf_ok, n, &r);
  if (s != TL_OK) return s;
  hipError_t e = launch(r, a, n, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "generated kernel launch");
  return TL_OK;
}

}  // namespace tl

extern "C" {

int tl_abi_version(void) { return TL_ABI_VERSION; }

const char* tl_last_error(void) { return g_last_error.c_str(); }

const char* tl_status_string(tl_status s) {
  switch (s) {
    case TL_OK: return "TL_OK";
    case TL_ERR_NULL: return "TL_ERR_NULL";
    case TL_ERR_SIZE: return "TL_ERR_SIZE";
    case TL_ERR_ALIAS: return "TL_ERR_ALIAS";
    case TL_ERR_ALIGN: return "TL_ERR_ALIGN";
    case TL_ERR_HIP: return "TL_ERR_HIP";
    case TL_ERR_INVALID: return "TL_ERR_INVALID";
    default: return "TL_ERR_UNKNOWN";
  }
}

tl_status tl_sym_inverse(int64_t n, tl_cfield g, tl_field ginv, void* stream, const tl_tune* tune) {
  if (n < 0) return fail(TL_ERR_SIZE, "n=%lld < 0", (long long)n);
  if (n == 0) return TL_OK;
  Checker c(n);
  c.field("g", g.ptr, g.ld, 6, false);
  c.field("ginv", ginv.ptr, ginv.ld, 6, true);
  if (c.overlaps() != TL_OK) return c.st;
  tl::KArgs a = zero_args();
  set_in(a, 0, g);
  set_out(a, 0, ginv);
  return run(tl::KernelId::SymInverse, c, tune, a, stream);
}

tl_status tl_christoffel(int64_t n, tl_cfield ginv, tl_cfield dg, tl_field gamma, void* stream,
                         const tl_tune* tune) {
  if (n < 0) return fail(TL_ERR_SIZE, "n=%lld < 0", (long long)n);
  if (n == 0) return TL_OK;
  Checker c(n);
  c.field("ginv", ginv.ptr, ginv.ld, 6, false);
  c.field("dg", dg.ptr, dg.ld, 18, false);
  c.field("gamma", gamma.ptr, gamma.ld, 18, true);
  if (c.overlaps() != TL_OK) return c.st;
  tl::KArgs a = zero_args();
  set_in(a, 0, ginv);
  set_in(a, 1, dg);
  set_out(a, 0, gamma);
  return run(tl::KernelId::Christoffel, c, tune, a, stream);
}

tl_status tl_cov_deriv(int64_t n, tl_cfield gamma, tl_cfield beta, tl_cfield dbeta,
                       tl_field nabla_beta, void* stream, const tl_tune* tune) {
  if (n < 0) return fail(TL_ERR_SIZE, "n=%lld < 0", (long long)n);
  if (n == 0) return TL_OK;
  Checker c(n);
  c.field("gamma", gamma.ptr, gamma.ld, 18, false);
  c.field("beta", beta.ptr, beta.ld, 3, false);
  c.field("dbeta", dbeta.ptr, dbeta.ld, 9, false);
  c.field("nabla_beta", nabla_beta.ptr, nabla_beta.ld, 9, true);
  if (c.overlaps() != TL_OK) return c.st;
  tl::KArgs a = zero_args();
  set_in(a, 0, gamma);
  set_in(a, 1, beta);
  set_in(a, 2, dbeta);
  set_out(a, 0, nabla_beta);
  return run(tl::KernelId::CovDeriv, c, tune, a, stream);
}

tl_status tl_dtg(int64_t n, tl_cfield alpha, tl_cfield K, tl_cfield nabla_beta, tl_field dtg,
                 void* stream, const tl_tune* tune) {
  if (n < 0) return fail(TL_ERR_SIZE, "n=%lld < 0", (long long)n);
  if (n == 0) return TL_OK;
  Checker c(n);
  c.field("alpha", alpha.ptr, alpha.ld, 1, false);
  c.field("K", K.ptr, K.ld, 6, false);
  c.field("nabla_beta", nabla_beta.ptr, nabla_beta.ld, 9, false);
  c.field("dtg", dtg.ptr, dtg.ld, 6, true);
  if (c.overlaps() != TL_OK) return c.st;
  tl::KArgs a = zero_args();
  set_in(a, 0, alpha);
  set_in(a, 1, K);
  set_in(a, 2, nabla_beta);
  set_out(a, 0, dtg);
  return run(tl::KernelId::Dtg, c, tune, a, stream);
}

static void chain_fields(Checker& c, tl_cfield g, tl_cfield dg, tl_cfield beta, tl_cfield dbeta,
                         tl_cfield K, tl_cfield alpha, tl_field dtg) {
  c.field("g", g.ptr, g.ld, 6, false);
  c.field("dg", dg.ptr, dg.ld, 18, false);
  c.field("beta", beta.ptr, beta.ld, 3, false);
  c.field("dbeta", dbeta.ptr, dbeta.ld, 9, false);
  c.field("K", K.ptr, K.ld, 6, false);
  c.field("alpha", alpha.ptr, alpha.ld, 1, false);
  c.field("dtg", dtg.ptr, dtg.ld, 6, true);
}

static tl::KArgs chain_args(tl_cfield g, tl_cfield dg, tl_cfield beta, tl_cfield dbeta, tl_cfield K,
                            tl_cfield alpha, tl_field dtg) {
  tl::KArgs a = zero_args();
  set_in(a, 0, g);
  set_in(a, 1, dg);
  set_in(a, 2, beta);
  set_in(a, 3, dbeta);
  set_in(a, 4, K);
  set_in(a, 5, alpha);
  a.ldin[5] = 0;
  set_out(a, 0, dtg);
  return a;
}

tl_status tl_dtg_chain(int64_t n, tl_cfield g, tl_cfield dg, tl_cfield beta, tl_cfield dbeta,
                       tl_cfield K, tl_cfield alpha, tl_field dtg, void* stream,
                       const tl_tune* tune) {
  if (n < 0) return fail(TL_ERR_SIZE, "n=%lld < 0", (long long)n);
  if (n == 0) return TL_OK;
  Checker c(n);
  chain_fields(c, g, dg, beta, dbeta, K, alpha, dtg);
  if (c.overlaps() != TL_OK) return c.st;
  return run(tl::KernelId::Chain, c, tune, chain_args(g, dg, beta, dbeta, K, alpha, dtg), stream);
}

static bool all_null(tl_field a, tl_field b, tl_field c, tl_field d, tl_field e, tl_field f) {
  return !a.ptr && !b.ptr && !c.ptr && !d.ptr && !e.ptr && !f.ptr;
}

static void bwd_fields(Checker& c, tl_cfield g, tl_cfield dg, tl_cfield beta, tl_cfield K,
                       tl_cfield alpha, tl_cfield w, tl_field g_bar, tl_field dg_bar,
                       tl_field beta_bar, tl_field dbeta_bar, tl_field K_bar, tl_field alpha_bar) {
  c.field("g", g.ptr, g.ld, 6, false);
  c.field("dg", dg.ptr, dg.ld, 18, false);
  c.field("beta", beta.ptr, beta.ld, 3, false);
  c.field("K", K.ptr, K.ld, 6, false);
  c.field("alpha", alpha.ptr, alpha.ld, 1, false);
  c.field("w", w.ptr, w.ld, 6, false);
  c.field("g_bar", g_bar.ptr, g_bar.ld, 6, true, true);
  c.field("dg_bar", dg_bar.ptr, dg_bar.ld, 18, true, true);
  c.field("beta_bar", beta_bar.ptr, beta_bar.ld, 3, true, true);
  c.field("dbeta_bar", dbeta_bar.ptr, dbeta_bar.ld, 9, true, true);
  c.field("K_bar", K_bar.ptr, K_bar.ld, 6, true, true);
  c.field("alpha_bar", alpha_bar.ptr, alpha_bar.ld, 1, true, true);
}

static tl::KArgs bwd_args(tl_cfield g, tl_cfield dg, tl_cfield beta, tl_cfield K,
                          tl_cfield alpha, tl_cfield w, tl_field g_bar, tl_field dg_bar,
                          tl_field beta_bar, tl_field dbeta_bar, tl_field K_bar,
                          tl_field alpha_bar) {
  tl::KArgs a = zero_args();
  set_in(a, 0, g);
  set_in(a, 1, dg);
  set_in(a, 2, beta);
  set_in(a, 3, K);
  set_in(a, 4, alpha);
  a.ldin[4] = 0;
  set_in(a, 5, w);
  set_out(a, 0, g_bar);
  set_out(a, 1, dg_bar);
  set_out(a, 2, beta_bar);
  set_out(a, 3, dbeta_bar);
  set_out(a, 4, K_bar);
  set_out(a, 5, alpha_bar);
  a.ldout[5] = 0;
  return a;
}

tl_status tl_dtg_chain_bwd(int64_t n, tl_cfield g, tl_cfield dg, tl_cfield beta, tl_cfield K,
                           tl_cfield alpha, tl_cfield w, tl_field g_bar, tl_field dg_bar,
                           tl_field beta_bar, tl_field dbeta_bar, tl_field K_bar,
                           tl_field alpha_bar, void* stream, const tl_tune* tune) {
  if (n < 0) return fail(TL_ERR_SIZE, "n=%lld < 0", (long long)n);
  if (n == 0) return TL_OK;
  if (all_null(g_bar, dg_bar, beta_bar, dbeta_bar, K_bar, alpha_bar))
    return fail(TL_ERR_NULL, "every gradient output is NULL");
  Checker c(n);
  bwd_fields(c, g, dg, beta, K, alpha, w, g_bar, dg_bar, beta_bar, dbeta_bar, K_bar, alpha_bar);
  if (c.overlaps() != TL_OK) return c.st;
  return run(tl::KernelId::ChainBwd, c, tune,
             bwd_args(g, dg, beta, K, alpha, w, g_bar, dg_bar, beta_bar, dbeta_bar, K_bar,
                      alpha_bar),
             stream);
}

tl_status tl_dtg_chain_fwd_bwd(int64_t n, tl_cfield g, tl_cfield dg, tl_cfield beta,
                           tl_cfield dbeta, tl_cfield K, tl_cfield alpha, tl_cfield w,
                           tl_field dtg, tl_field g_bar, tl_field dg_bar, tl_field beta_bar,
                           tl_field dbeta_bar, tl_field K_bar, tl_field alpha_bar, void* stream,
                           const tl_tune* tune) {
  if (n < 0) return fail(TL_ERR_SIZE, "n=%lld < 0", (long long)n);
  if (n == 0) return TL_OK;
  if (!dtg.ptr && !g_bar.ptr && !dg_bar.ptr && !beta_bar.ptr && !dbeta_bar.ptr && !K_bar.ptr &&
      !alpha_bar.ptr)
    return fail(TL_ERR_NULL, "every output is NULL");
  Checker c(n);
  c.field("g", g.ptr, g.ld, 6, false);
  c.field("dg", dg.ptr, dg.ld, 18, false);
  c.field("beta", beta.ptr, beta.ld, 3, false);
  c.field("dbeta", dbeta.ptr, dbeta.ld, 9, false);
  c.field("K", K.ptr, K.ld, 6, false);
  c.field("alpha", alpha.ptr, alpha.ld, 1, false);
  c.field("w", w.ptr, w.ld, 6, false);
  c.field("dtg", dtg.ptr, dtg.ld, 6, true, true);
  c.field("g_bar", g_bar.ptr, g_bar.ld, 6, true, true);
  c.field("dg_bar", dg_bar.ptr, dg_bar.ld, 18, true, true);
  c.field("beta_bar", beta_bar.ptr, beta_bar.ld, 3, true, true);
  c.field("dbeta_bar", dbeta_bar.ptr, dbeta_bar.ld, 9, true, true);
  c.field("K_bar", K_bar.ptr, K_bar.ld, 6, true, true);
  c.field("alpha_bar", alpha_bar.ptr, alpha_bar.ld, 1, true, true);
  if (c.overlaps() != TL_OK) return c.st;
  tl::KArgs a = zero_args();
  set_in(a, 0, g);
  set_in(a, 1, dg);
  set_in(a, 2, beta);
  set_in(a, 3, dbeta);
  set_in(a, 4, K);
  set_in(a, 5, alpha);
  a.ldin[5] = 0;
  set_in(a, 6, w);
  set_out(a, 0, dtg);
  set_out(a, 1, g_bar);
  set_out(a, 2, dg_bar);
  set_out(a, 3, beta_bar);
  set_out(a, 4, dbeta_bar);
  set_out(a, 5, K_bar);
  set_out(a, 6, alpha_bar);
  a.ldout[6] = 0;
  return run(tl::KernelId::ChainFwdBwd, c, tune, a, stream);
}

namespace {
// Input component counts (0-terminated) and output count of each expression.
const int kExprIn[TL_EXPR_COUNT][5] = {{3}, {9}, {27}, {3, 3}, {3, 3, 3}, {3, 3, 3, 3}, {3, 3},
                                       {3, 3, 3}, {3, 3, 3, 3}, {9, 81}, {9, 9, 81},
                                       {9, 9, 9, 81}, {1, 6, 3}};
const int kExprOut[TL_EXPR_COUNT] = {3, 9, 27, 3, 3, 3, 9, 27, 81, 81, 81, 81, 6};
const char* const kExprName[TL_EXPR_COUNT] = {
    "assign1", "assign2", "assign3", "add1", "add2", "add3", "mult1",
    "mult2", "mult3", "contract1", "contract2", "contract3", "kij"};
int expr_nin(int id) {
  int k = 0;
  while (k < 4 && kExprIn[id][k] > 0) ++k;
  return k;
}
}  // namespace

tl_status tl_expr_shape(int32_t expr, int32_t* nin, int32_t* in_ncomp, int32_t* out_ncomp) {
  if (expr < 0 || expr >= TL_EXPR_COUNT) return fail(TL_ERR_INVALID, "unknown expression %d", expr);
  const int k = expr_nin(expr);
  if (nin) *nin = k;
  if (in_ncomp)
    for (int f = 0; f < k; ++f) in_ncomp[f] = kExprIn[expr][f];
  if (out_ncomp) *out_ncomp = kExprOut[expr];
  return TL_OK;
}

tl_status tl_expr(int32_t expr, int64_t n, const tl_cfield* in, int32_t nin, tl_field out,
                  void* stream, const tl_tune* tune) {
  if (expr < 0 || expr >= TL_EXPR_COUNT) return fail(TL_ERR_INVALID, "unknown expression %d", expr);
  const int k = expr_nin(expr);
  if (nin != k) return fail(TL_ERR_INVALID, "%s takes %d inputs, got %d", kExprName[expr], k, nin);
  if (n < 0) return fail(TL_ERR_SIZE, "n=%lld < 0", (long long)n);
  if (n == 0) return TL_OK;
  if (in == nullptr) return fail(TL_ERR_NULL, "in is NULL");
  static const char* const names[4] = {"in[0]", "in[1]", "in[2]", "in[3]"};
  Checker c(n);
  for (int f = 0; f < k; ++f) c.field(names[f], in[f].ptr, in[f].ld, kExprIn[expr][f], false);
  c.field("out", out.ptr, out.ld, kExprOut[expr], true);
  if (c.overlaps() != TL_OK) return c.st;
  tl::KArgs a = zero_args();
  for (int f = 0; f < k; ++f) set_in(a, f, in[f]);
  set_out(a, 0, out);
  tl::Resolved r;
  tl_status s = resolve(tl::KernelId::Generic, tune, c.vec_ok, c.buf_ok, n, &r);
  if (s != TL_OK) return s;
  hipError_t e = tl::launch_expr(expr, r, a, n, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "expression launch");
  return TL_OK;
}

tl_status tl_bw_twin(int64_t n, int32_t nin, tl_cfield in, int32_t nout, tl_field out, void* stream,
                     const tl_tune* tune) {
  bool known = false;
#define TL_TWIN(I, O) known = known || (nin == I && nout == O);
  TL_TWIN_SHAPES(TL_TWIN)
#undef TL_TWIN
  if (!known) return fail(TL_ERR_INVALID, "no twin for %d reads and %d writes", nin, nout);
  if (n < 0) return fail(TL_ERR_SIZE, "n=%lld < 0", (long long)n);
  if (n == 0) return TL_OK;
  Checker c(n);
  c.field("in", in.ptr, in.ld, nin, false);
  c.field("out", out.ptr, out.ld, nout, true);
  if (c.overlaps() != TL_OK) return c.st;
  tl::KArgs a = zero_args();
  set_in(a, 0, in);
  set_out(a, 0, out);
  tl::Resolved r;
  tl_status s = resolve(tl::KernelId::Generic, tune, c.vec_ok, c.buf_ok, n, &r);
  if (s != TL_OK) return s;
  hipError_t e = tl::launch_twin(nin, nout, r, a, n, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "twin launch");
  return TL_OK;
}

tl_status tl_bw_copy(int64_t n, const double* src, double* dst, void* stream) {
  if (n < 0) return fail(TL_ERR_SIZE, "n=%lld < 0", (long long)n);
  if (n == 0) return TL_OK;
  Checker c(n);
  c.field("src", src, n, 1, false);
  c.field("dst", dst, n, 1, true);
  if (c.overlaps() != TL_OK) return c.st;
  int64_t grid = (n + 511) / 512;
  if (grid > (1 << 20)) grid = 1 << 20;
  hipError_t e = tl::launch_copy(src, dst, n, grid, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "copy launch");
  return TL_OK;
}

tl_status tl_bw_stream(int64_t n, int32_t kind, const double* src, double* dst, void* stream) {
  if (kind != TL_BW_READ && kind != TL_BW_WRITE)
    return fail(TL_ERR_INVALID, "kind=%d is neither TL_BW_READ nor TL_BW_WRITE", kind);
  if (n < 0) return fail(TL_ERR_SIZE, "n=%lld < 0", (long long)n);
  if (n == 0) return TL_OK;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e;
  if (kind == TL_BW_READ) {
    Checker c(n);
    c.field("src", src, n, 1, false);
    if (c.st != TL_OK) return c.st;
    Checker p(TL_BW_READ_BLOCKS);
    p.field("partial", dst, TL_BW_READ_BLOCKS, 1, true);
    if (p.st != TL_OK) return p.st;
    c.spans.insert(c.spans.end(), p.spans.begin(), p.spans.end());
    if (c.overlaps() != TL_OK) return c.st;
    int64_t grid = (n + 511) / 512;
    if (grid > TL_BW_READ_BLOCKS) grid = TL_BW_READ_BLOCKS;
    e = tl::launch_read(src, dst, n, grid, reinterpret_cast<uintptr_t>(src) % 16 == 0, s);
  } else {
    Checker c(n);
    c.field("dst", dst, n, 1, true);
    if (c.st != TL_OK) return c.st;
    int64_t grid = (n + 511) / 512;
    if (grid > 32768) grid = 32768;
    e = tl::launch_write(dst, n, grid, reinterpret_cast<uintptr_t>(dst) % 16 == 0, s);
  }
  if (e != hipSuccess) return hip_fail(e, "bandwidth reference launch");
  return TL_OK;
}

// ---------------------------------------------------------------- batch plans

namespace {

// What a plan is built from: each domain's n and kernel arguments, the spans
// of all its fields (already validated per domain) and the layout facts.
struct PlanInput {
  std::vector<int64_t> n;
  std::vector<tl::KArgs> args;
  std::vector<Span> spans;
  bool vec_ok = true, buf_ok = true;
  int64_t points = 0;
  void add(int64_t nd, const tl::KArgs& a, const Checker& c) {
    n.push_back(nd);
    args.push_back(a);
    if (nd == 0) return;
    spans.insert(spans.end(), c.spans.begin(), c.spans.end());
    vec_ok = vec_ok && c.vec_ok;
    buf_ok = buf_ok && c.buf_ok;
    points += nd;
  }
};

// The host side of a batched launch: the resolved shape, the device-layout
// domain table, the tile prefix sums and the tile -> subgrid map, and the
// grid (one block per tile, or a persistent grid of grid_mult blocks per
// compute unit, each block walking one contiguous chunk of tiles).
struct PlanTables {
  tl::Resolved r;
  std::vector<tl::BatchDomain> doms;
  std::vector<int64_t> start;
  std::vector<int32_t> tile_dom;
  int64_t points = 0, ntiles = 0, grid = 0, chunk = 1;
};

// Checks the outputs of all domains against every field of every domain and
// builds the tables (the tile -> domain map only if tile_map).
tl_status plan_tables(tl::KernelId kid, PlanInput& in, const tl_tune* tune, PlanTables* t,
                      bool tile_map = true) {
  {
    const char* a = nullptr;
    const char* b = nullptr;
    if (Checker::overlapping(in.spans, &a, &b))
      return fail(TL_ERR_ALIAS, "%s of one domain overlaps %s of another", a, b);
  }
  tl_status s = resolve(kid, tune, in.vec_ok, in.buf_ok, in.points, &t->r);
  if (s != TL_OK) return s;
  const tl::Resolved& r = t->r;
  const int32_t ndom = static_cast<int32_t>(in.n.size());
  t->doms.assign(ndom, tl::BatchDomain{});
  t->start.assign(ndom + 1, 0);
  t->tile_dom.clear();
  const int64_t per = static_cast<int64_t>(r.block) * r.ppt;
  for (int32_t d = 0; d < ndom; ++d) {
    std::memset(&t->doms[d], 0, sizeof(tl::BatchDomain));
    t->doms[d].n = in.n[d];
    if (in.n[d] > 0) t->doms[d].args = in.args[d];
    t->start[d + 1] = t->start[d] + (in.n[d] + per - 1) / per;
    if (tile_map)
      t->tile_dom.insert(t->tile_dom.end(), static_cast<size_t>(t->start[d + 1] - t->start[d]), d);
  }
  t->points = in.points;
  t->ntiles = t->start[ndom];
  int64_t blocks = t->ntiles;
  if (r.grid_mult > 0) blocks = static_cast<int64_t>(r.grid_mult) * r.num_cu;
  if (r.xcd) blocks = (blocks + 7) & ~static_cast<int64_t>(7);
  if (blocks < 1) blocks = 1;
  t->chunk = (t->ntiles + blocks - 1) / blocks;
  if (t->chunk < 1) t->chunk = 1;
  t->grid = (t->ntiles + t->chunk - 1) / t->chunk;
  if (r.xcd) t->grid = (t->grid + 7) & ~static_cast<int64_t>(7);
  if (t->grid < 1) t->grid = 1;
  return TL_OK;
}

// Builds the tables, copies them to the device and captures the launch.
tl_status build_plan(tl::KernelId kid, PlanInput& in, const tl_tune* tune, tl_batch_plan** out) {
  PlanTables t;
  tl_status s = plan_tables(kid, in, tune, &t);
  if (s != TL_OK) return s;
  const int32_t ndom = static_cast<int32_t>(t.doms.size());
  tl_batch_plan* p = new (std::nothrow) tl_batch_plan;
  if (p == nullptr) return fail(TL_ERR_INVALID, "out of host memory");
  p->kid = kid;
  p->r = t.r;
  p->ndom = ndom;
  p->points = t.points;
  p->ntiles = t.ntiles;
  p->grid = t.grid;
  p->chunk = t.chunk;
  hipError_t e = hipGetDevice(&p->device);
  auto cleanup = [&](hipError_t err, const char* what) {
    tl_status st = hip_fail(err, what);
    tl_batch_plan_destroy(p);
    return st;
  };
  if (e != hipSuccess) return cleanup(e, "hipGetDevice");
  e = hipMalloc(reinterpret_cast<void**>(&p->d_doms), sizeof(tl::BatchDomain) * ndom);
  if (e != hipSuccess) return cleanup(e, "hipMalloc(domains)");
  e = hipMalloc(reinterpret_cast<void**>(&p->d_start), sizeof(int64_t) * (ndom + 1));
  if (e != hipSuccess) return cleanup(e, "hipMalloc(tile starts)");
  e = hipMemcpy(p->d_doms, t.doms.data(), sizeof(tl::BatchDomain) * ndom, hipMemcpyHostToDevice);
  if (e != hipSuccess) return cleanup(e, "hipMemcpy(domains)");
  e = hipMemcpy(p->d_start, t.start.data(), sizeof(int64_t) * (ndom + 1), hipMemcpyHostToDevice);
  if (e != hipSuccess) return cleanup(e, "hipMemcpy(tile starts)");
  if (p->ntiles > 0) {
    e = hipMalloc(reinterpret_cast<void**>(&p->d_tile_dom), sizeof(int32_t) * p->ntiles);
    if (e != hipSuccess) return cleanup(e, "hipMalloc(tile table)");
    e = hipMemcpy(p->d_tile_dom, t.tile_dom.data(), sizeof(int32_t) * p->ntiles,
                  hipMemcpyHostToDevice);
    if (e != hipSuccess) return cleanup(e, "hipMemcpy(tile table)");
  }
  if (p->ntiles > 0) {
    e = hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking);
    if (e != hipSuccess) return cleanup(e, "hipStreamCreate");
    e = hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return cleanup(e, "hipStreamBeginCapture");
    hipError_t le = tl::launch_batched(p->kid, p->r, p->d_doms, p->d_start, p->d_tile_dom,
                                       p->ntiles, p->grid, p->chunk, p->cap);
    e = hipStreamEndCapture(p->cap, &p->graph);
    if (le != hipSuccess) return cleanup(le, "captured launch");
    if (e != hipSuccess) return cleanup(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return cleanup(e, "hipGraphInstantiate");
  }
  *out = p;
  return TL_OK;
}

tl_status plan_preamble(const void* doms, int32_t ndom, tl_batch_plan** out) {
  if (out == nullptr) return fail(TL_ERR_NULL, "out is NULL");
  *out = nullptr;
  if (doms == nullptr) return fail(TL_ERR_NULL, "doms is NULL");
  if (ndom < 1) return fail(TL_ERR_SIZE, "ndom=%d < 1", ndom);
  return TL_OK;
}

}  // namespace

// Validates every domain of a forward batch (as tl_dtg_chain would) and
// collects their arguments and field spans.
static tl_status chain_domains(const tl_domain* doms, int32_t ndom, PlanInput* in) {
  for (int32_t d = 0; d < ndom; ++d) {
    const tl_domain& x = doms[d];
    if (x.n < 0) return fail(TL_ERR_SIZE, "domain %d: n=%lld < 0", d, (long long)x.n);
    Checker c(x.n);
    if (x.n > 0) {
      chain_fields(c, x.g, x.dg, x.beta, x.dbeta, x.K, x.alpha, x.dtg);
      if (c.overlaps() != TL_OK) return fail(c.st, "domain %d: %s", d, g_last_error.c_str());
    }
    in->add(x.n, x.n > 0 ? chain_args(x.g, x.dg, x.beta, x.dbeta, x.K, x.alpha, x.dtg)
                         : zero_args(), c);
  }
  return TL_OK;
}

tl_status tl_batch_plan_create(const tl_domain* doms, int32_t ndom, const tl_tune* tune,
                               tl_batch_plan** out) {
  const tl_status s0 = plan_preamble(doms, ndom, out);
  if (s0 != TL_OK) return s0;
  PlanInput in;
  const tl_status s1 = chain_domains(doms, ndom, &in);
  if (s1 != TL_OK) return s1;
  return build_plan(tl::KernelId::ChainBatched, in, tune, out);
}

tl_status tl_batch_run_noalloc(const tl_domain* doms, int32_t ndom, const tl_tune* tune,
                               void* stream) {
  if (doms == nullptr) return fail(TL_ERR_NULL, "doms is NULL");
  if (ndom < 1 || ndom > TL_NOALLOC_MAX_DOMAINS)
    return fail(TL_ERR_SIZE, "ndom=%d not in [1, %d] (TL_NOALLOC_MAX_DOMAINS)", ndom,
                TL_NOALLOC_MAX_DOMAINS);
  PlanInput in;
  const tl_status s1 = chain_domains(doms, ndom, &in);
  if (s1 != TL_OK) return s1;
  PlanTables t;
  const tl_status s2 = plan_tables(tl::KernelId::ChainBatched, in, tune, &t, false);
  if (s2 != TL_OK) return s2;
  if (t.ntiles > TL_NOALLOC_MAX_TILES)
    return fail(TL_ERR_SIZE,
                "%lld tiles of %d points exceed TL_NOALLOC_MAX_TILES=%d (a larger block or ppt "
                "takes fewer tiles; a batch plan has no such limit)",
                (long long)t.ntiles, t.r.block * t.r.ppt, TL_NOALLOC_MAX_TILES);
  hipError_t e = tl::launch_batched_noalloc(t.r, t.doms.data(), t.start.data(), ndom, t.ntiles,
                                            t.grid, t.chunk, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "no-allocation batched launch");
  return TL_OK;
}

tl_status tl_batch_plan_bwd_create(const tl_domain_bwd* doms, int32_t ndom, const tl_tune* tune,
                                   tl_batch_plan** out) {
  const tl_status s0 = plan_preamble(doms, ndom, out);
  if (s0 != TL_OK) return s0;
  PlanInput in;
  for (int32_t d = 0; d < ndom; ++d) {
    const tl_domain_bwd& x = doms[d];
    if (x.n < 0) return fail(TL_ERR_SIZE, "domain %d: n=%lld < 0", d, (long long)x.n);
    Checker c(x.n);
    if (x.n > 0) {
      if (all_null(x.g_bar, x.dg_bar, x.beta_bar, x.dbeta_bar, x.K_bar, x.alpha_bar))
        return fail(TL_ERR_NULL, "domain %d: every gradient output is NULL", d);
      bwd_fields(c, x.g, x.dg, x.beta, x.K, x.alpha, x.w, x.g_bar, x.dg_bar, x.beta_bar,
                 x.dbeta_bar, x.K_bar, x.alpha_bar);
      if (c.overlaps() != TL_OK) return fail(c.st, "domain %d: %s", d, g_last_error.c_str());
    }
    in.add(x.n,
           x.n > 0 ? bwd_args(x.g, x.dg, x.beta, x.K, x.alpha, x.w, x.g_bar, x.dg_bar,
                              x.beta_bar, x.dbeta_bar, x.K_bar, x.alpha_bar)
                   : zero_args(),
           c);
  }
  return build_plan(tl::KernelId::ChainBwdBatched, in, tune, out);
}

static tl_status plan_device_check(const tl_batch_plan* p) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != p->device)
    return fail(TL_ERR_INVALID, "plan belongs to device %d, current device is %d", p->device, dev);
  return TL_OK;
}

tl_status tl_batch_plan_launch(tl_batch_plan* p, void* stream) {
  if (p == nullptr) return fail(TL_ERR_NULL, "plan is NULL");
  if (plan_device_check(p) != TL_OK) return TL_ERR_INVALID;
  if (p->ntiles == 0) return TL_OK;
  hipError_t e = hipGraphLaunch(p->exec, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  return TL_OK;
}

tl_status tl_batch_plan_launch_direct(tl_batch_plan* p, void* stream) {
  if (p == nullptr) return fail(TL_ERR_NULL, "plan is NULL");
  if (plan_device_check(p) != TL_OK) return TL_ERR_INVALID;
  if (p->ntiles == 0) return TL_OK;
  hipError_t e = tl::launch_batched(p->kid, p->r, p->d_doms, p->d_start, p->d_tile_dom,
                                    p->ntiles, p->grid, p->chunk, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "batched launch");
  return TL_OK;
}

tl_status tl_batch_plan_info(const tl_batch_plan* p, int64_t* points, int64_t* tiles,
                             int64_t* blocks) {
  if (p == nullptr) return fail(TL_ERR_NULL, "plan is NULL");
  if (points) *points = p->points;
  if (tiles) *tiles = p->ntiles;
  if (blocks) *blocks = p->grid;
  return TL_OK;
}

tl_status tl_batch_plan_destroy(tl_batch_plan* p) {
  if (p == nullptr) return TL_OK;
  hipError_t first = hipSuccess;
  auto keep = [&](hipError_t e) {
    if (first == hipSuccess && e != hipSuccess) first = e;
  };
  // Work on the plan's device (the caller's current device may differ), and
  // wait for its launches before freeing what they read.
  int prev = -1;
  keep(hipGetDevice(&prev));
  const bool switched = prev >= 0 && prev != p->device;
  if (switched) keep(hipSetDevice(p->device));
  if (p->d_doms || p->d_start || p->d_tile_dom || p->exec) keep(hipDeviceSynchronize());
  if (p->exec) keep(hipGraphExecDestroy(p->exec));
  if (p->graph) keep(hipGraphDestroy(p->graph));
  if (p->cap) keep(hipStreamDestroy(p->cap));
  if (p->d_doms) keep(hipFree(p->d_doms));
  if (p->d_start) keep(hipFree(p->d_start));
  if (p->d_tile_dom) keep(hipFree(p->d_tile_dom));
  if (switched) keep(hipSetDevice(prev));
  delete p;
  if (first != hipSuccess) return hip_fail(first, "plan destroy");
  return TL_OK;
}

// ---------------------------------------------------------------- introspection

tl_status tl_kernel_info(const char* kernel, const tl_tune* tune, tl_kernel_attr* out) {
  if (kernel == nullptr || out == nullptr) return fail(TL_ERR_NULL, "kernel or out is NULL");
  static const struct {
    const char* name;
    tl::KernelId id;
  } names[] = {{"sym_inverse", tl::KernelId::SymInverse}, {"christoffel", tl::KernelId::Christoffel},
               {"cov_deriv", tl::KernelId::CovDeriv},     {"dtg", tl::KernelId::Dtg},
               {"dtg_chain", tl::KernelId::Chain},        {"dtg_chain_bwd", tl::KernelId::ChainBwd},
               {"dtg_chain_batched", tl::KernelId::ChainBatched},
               {"dtg_chain_fwd_bwd", tl::KernelId::ChainFwdBwd},
               {"dtg_chain_bwd_batched", tl::KernelId::ChainBwdBatched}};
  const tl::KernelId* id = nullptr;
  for (const auto& x : names)
    if (std::strcmp(x.name, kernel) == 0) id = &x.id;
  int expr = -1;
  for (int e = 0; e < TL_EXPR_COUNT; ++e)
    if (std::strcmp(kExprName[e], kernel) == 0) expr = e;
  if (id == nullptr && expr < 0) return fail(TL_ERR_INVALID, "unknown kernel '%s'", kernel);
  tl::Resolved r;
  tl_status s = resolve(id ? *id : tl::KernelId::Generic, tune, true, true, int64_t(1) << 24, &r);
  if (s != TL_OK) return s;
  const void* fn = id ? tl::kernel_address(*id, r) : tl::expr_address(expr, r);
  if (fn == nullptr) return fail(TL_ERR_INVALID, "no instantiation for this tuning");
  hipFuncAttributes attr;
  hipError_t e = hipFuncGetAttributes(&attr, fn);
  if (e != hipSuccess) return hip_fail(e, "hipFuncGetAttributes");
  // The block size the kernel actually runs with (a wide body caps it).
  const int block = std::min(r.block, attr.maxThreadsPerBlock);
  int blocks_per_cu = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks_per_cu, fn, block, 0);
  if (e != hipSuccess) return hip_fail(e, "hipOccupancyMaxActiveBlocksPerMultiprocessor");
  tl::KernelResources res{-1, -1, -1, -1, -1};
  tl::kernel_resources(hipKernelNameRefByPtr(fn, nullptr), &res);
  out->block = block;
  out->ppt = id ? r.ppt : tl::expr_ppt(expr, r.ppt);
  out->flags = (r.nt ? TL_TUNE_NT : 0) | (r.xcd ? TL_TUNE_XCD : 0);
  out->vgprs = attr.numRegs;
  out->agprs = res.agprs;
  out->sgprs = res.sgprs;
  out->scratch_bytes = static_cast<int32_t>(attr.localSizeBytes);
  // four SIMDs per compute unit, 64-wide waves
  out->waves_per_simd = blocks_per_cu * ((block + 63) / 64) / 4;
  out->max_waves_per_simd = res.waves_per_simd;
  out->max_threads = attr.maxThreadsPerBlock;
  return TL_OK;
}

}  // extern "C"
