// Test driver for the C ABI without Python or torch: device buffers from
// hipMalloc, the fused chain, its adjoint and both in one pass on a stream of
// its own, an unfused step, batch plans, the batch without allocation, and
// argument errors; every result is compared on
// the host with the CPU oracle (liboracle.so), per component, relative to the
// component's largest magnitude, against 1e-12.  Exit status 0 means every
// check passed.  Test infrastructure: built by the package build next to the
// oracle, run by tests/test_gpu_c_abi.py.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <string_view>
#include <vector>

#include "tl.h"

extern "C" {
void tlo_dtg_chain(int64_t n, const double* g, const double* dg, const double* beta,
                   const double* dbeta, const double* K, const double* alpha, double* dtg);
void tlo_dtg_chain_vjp(int64_t n, const double* g, const double* dg, const double* beta,
                       const double* dbeta, const double* K, const double* alpha, const double* W,
                       double* g_bar, double* dg_bar, double* beta_bar, double* dbeta_bar,
                       double* K_bar, double* alpha_bar);
void tlo_sym_inverse(int64_t n, const double* g, double* ginv);
}

namespace {

int failures = 0;

void expect(bool ok, const char* what) {
  if (!ok) {
    std::printf("FAIL %s\n", what);
    ++failures;
  }
}

// splitmix64: a seeded source of test values (no arithmetic of the method).
struct Rng {
  uint64_t s;
  double uniform(double lo, double hi) {
    uint64_t z = (s += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z ^= z >> 31;
    return lo + (hi - lo) * static_cast<double>(z >> 11) * (1.0 / 9007199254740992.0);
  }
};

// Per-component relative error of x against r ([ncomp][n], both).
double rel_err(const std::vector<double>& x, const std::vector<double>& r, int ncomp, int64_t n) {
  double worst = 0.0;
  for (int c = 0; c < ncomp; ++c) {
    double scale = 0.0, diff = 0.0;
    for (int64_t p = 0; p < n; ++p) {
      scale = std::fmax(scale, std::fabs(r[c * n + p]));
      const double d = std::fabs(x[c * n + p] - r[c * n + p]);
      diff = std::isnan(d) ? INFINITY : std::fmax(diff, d);
    }
    worst = std::fmax(worst, diff / (scale > 0.0 ? scale : 1.0));
  }
  return worst;
}

struct Dev {
  double* p = nullptr;
  size_t count = 0;
  explicit Dev(size_t c) : count(c) {
    if (hipMalloc(reinterpret_cast<void**>(&p), c * sizeof(double)) != hipSuccess) p = nullptr;
  }
  ~Dev() {
    if (p) (void)hipFree(p);
  }
  void put(const std::vector<double>& h) {
    (void)hipMemcpy(p, h.data(), count * sizeof(double), hipMemcpyHostToDevice);
  }
  std::vector<double> get() const {
    std::vector<double> h(count);
    (void)hipMemcpy(h.data(), p, count * sizeof(double), hipMemcpyDeviceToHost);
    return h;
  }
};

}  // namespace

int main() {
  const int64_t n = 20011;  // several tiles and a ragged tail
  Rng rng{20240601ull};
  const int nc[7] = {6, 18, 3, 9, 6, 1, 6};  // g, dg, beta, dbeta, K, alpha, W
  std::vector<std::vector<double>> h(7);
  for (int f = 0; f < 7; ++f) h[f].resize(nc[f] * n);
  for (int64_t p = 0; p < n; ++p) {
    for (int c = 0; c < 6; ++c) h[0][c * n + p] = 0.1 * rng.uniform(-1.0, 1.0);
    h[0][0 * n + p] += 1.0;
    h[0][3 * n + p] += 1.0;
    h[0][5 * n + p] += 1.0;
  }
  for (auto& x : h[1]) x = rng.uniform(-1.0, 1.0);
  for (auto& x : h[2]) x = rng.uniform(-0.5, 0.5);
  for (auto& x : h[3]) x = rng.uniform(-2.0, 2.0);
  for (auto& x : h[4]) x = rng.uniform(-1.0, 1.0);
  for (auto& x : h[5]) x = rng.uniform(0.5, 1.5);
  for (auto& x : h[6]) x = rng.uniform(-2.0, 2.0);

  std::vector<Dev*> d;
  for (int f = 0; f < 7; ++f) {
    d.push_back(new Dev(nc[f] * n));
    expect(d[f]->p != nullptr, "hipMalloc input");
    d[f]->put(h[f]);
  }
  auto cf = [&](int f) { return tl_cfield{d[f]->p, n}; };
  hipStream_t s;
  expect(hipStreamCreate(&s) == hipSuccess, "hipStreamCreate");

  // forward
  Dev dtg(6 * n);
  expect(tl_dtg_chain(n, cf(0), cf(1), cf(2), cf(3), cf(4), cf(5), tl_field{dtg.p, n}, s,
                      nullptr) == TL_OK, "tl_dtg_chain status");
  // adjoint
  const int gc[6] = {6, 18, 3, 9, 6, 1};
  std::vector<Dev*> gb;
  for (int f = 0; f < 6; ++f) gb.push_back(new Dev(gc[f] * n));
  expect(tl_dtg_chain_bwd(n, cf(0), cf(1), cf(2), cf(4), cf(5), cf(6), tl_field{gb[0]->p, n},
                          tl_field{gb[1]->p, n}, tl_field{gb[2]->p, n}, tl_field{gb[3]->p, n},
                          tl_field{gb[4]->p, n}, tl_field{gb[5]->p, n}, s, nullptr) == TL_OK,
         "tl_dtg_chain_bwd status");
  // both in one pass, with a supplied launch shape
  Dev dtg2(6 * n);
  std::vector<Dev*> gb2;
  for (int f = 0; f < 6; ++f) gb2.push_back(new Dev(gc[f] * n));
  const tl_tune tune = {128, 1, TL_TUNE_NT | TL_TUNE_XCD, 0};
  expect(tl_dtg_chain_fwd_bwd(n, cf(0), cf(1), cf(2), cf(3), cf(4), cf(5), cf(6),
                              tl_field{dtg2.p, n}, tl_field{gb2[0]->p, n},
                              tl_field{gb2[1]->p, n}, tl_field{gb2[2]->p, n},
                              tl_field{gb2[3]->p, n}, tl_field{gb2[4]->p, n},
                              tl_field{gb2[5]->p, n}, s, &tune) == TL_OK,
         "tl_dtg_chain_fwd_bwd status");
  // an unfused step
  Dev ginv(6 * n);
  expect(tl_sym_inverse(n, cf(0), tl_field{ginv.p, n}, s, nullptr) == TL_OK,
         "tl_sym_inverse status");
  expect(hipStreamSynchronize(s) == hipSuccess, "hipStreamSynchronize");

  std::vector<double> ref(6 * n);
  tlo_dtg_chain(n, h[0].data(), h[1].data(), h[2].data(), h[3].data(), h[4].data(), h[5].data(),
                ref.data());
  std::vector<std::vector<double>> rg(6);
  for (int f = 0; f < 6; ++f) rg[f].resize(gc[f] * n);
  tlo_dtg_chain_vjp(n, h[0].data(), h[1].data(), h[2].data(), h[3].data(), h[4].data(),
                    h[5].data(), h[6].data(), rg[0].data(), rg[1].data(), rg[2].data(),
                    rg[3].data(), rg[4].data(), rg[5].data());
  std::vector<double> rinv(6 * n);
  tlo_sym_inverse(n, h[0].data(), rinv.data());

  double e = rel_err(dtg.get(), ref, 6, n);
  std::printf("dtg_chain rel err %.3e\n", e);
  expect(e <= 1e-12, "dtg_chain vs oracle");
  e = rel_err(dtg2.get(), ref, 6, n);
  expect(e <= 1e-12, "fwd_bwd d_t g vs oracle");
  for (int f = 0; f < 6; ++f) {
    e = rel_err(gb[f]->get(), rg[f], gc[f], n);
    std::printf("gradient %d rel err %.3e\n", f, e);
    expect(e <= 1e-12, "adjoint vs oracle");
    e = rel_err(gb2[f]->get(), rg[f], gc[f], n);
    expect(e <= 1e-12, "fwd_bwd gradient vs oracle");
  }
  e = rel_err(ginv.get(), rinv, 6, n);
  expect(e <= 1e-12, "sym_inverse vs oracle");

  // a batch plan over three subgrids that are point ranges of the same fields
  // ([0, 5000), [5000, 5001) and [7000, 20011)), inputs and outputs alike: the
  // outputs interleave in one buffer without sharing an element
  {
    const int64_t lo[3] = {0, 5000, 7000}, cnt[3] = {5000, 1, n - 7000};
    Dev outb(6 * n);
    std::vector<double> fill(6 * n, -7.0);
    outb.put(fill);
    tl_domain doms[3];
    for (int k = 0; k < 3; ++k) {
      auto sub = [&](int f) { return tl_cfield{d[f]->p + lo[k], n}; };
      doms[k] = tl_domain{cnt[k], sub(0), sub(1), sub(2), sub(3), sub(4), sub(5),
                          tl_field{outb.p + lo[k], n}};
    }
    tl_batch_plan* plan = nullptr;
    expect(tl_batch_plan_create(doms, 3, nullptr, &plan) == TL_OK && plan != nullptr,
           "tl_batch_plan_create");
    if (plan) {
      expect(tl_batch_plan_launch(plan, s) == TL_OK, "tl_batch_plan_launch");
      expect(hipStreamSynchronize(s) == hipSuccess, "plan sync");
      const std::vector<double> got = outb.get();
      std::vector<double> want(6 * n);
      bool untouched = true;
      for (int c = 0; c < 6; ++c)
        for (int64_t p = 0; p < n; ++p) {
          const bool in_domain = p < 5001 || p >= 7000;
          want[c * n + p] = in_domain ? ref[c * n + p] : -7.0;
          if (!in_domain && got[c * n + p] != -7.0) untouched = false;
        }
      e = rel_err(got, want, 6, n);
      std::printf("batch plan rel err %.3e\n", e);
      expect(e <= 1e-12, "batch plan vs oracle");
      expect(untouched, "points outside every subgrid untouched");
      expect(tl_batch_plan_destroy(plan) == TL_OK, "tl_batch_plan_destroy");
      // the same subgrids without allocating: bitwise the plan's result
      Dev outn(6 * n);
      outn.put(fill);
      tl_domain ndoms[3];
      for (int k = 0; k < 3; ++k) {
        ndoms[k] = doms[k];
        ndoms[k].dtg.ptr = outn.p + lo[k];
      }
      expect(tl_batch_run_noalloc(ndoms, 3, nullptr, s) == TL_OK, "tl_batch_run_noalloc");
      expect(hipStreamSynchronize(s) == hipSuccess, "no-allocation sync");
      expect(outn.get() == got, "no-allocation batch equals the plan bitwise");
      expect(tl_batch_run_noalloc(ndoms, TL_NOALLOC_MAX_DOMAINS + 1, nullptr, s) == TL_ERR_SIZE,
             "no-allocation batch refuses too many subgrids");
    }
    // two subgrids sharing an output element are refused
    tl_domain clash[2] = {doms[0], doms[0]};
    clash[1].n = 10;
    clash[1].dtg.ptr = outb.p + 4995;
    tl_batch_plan* bad = nullptr;
    expect(tl_batch_plan_create(clash, 2, nullptr, &bad) == TL_ERR_ALIAS && bad == nullptr,
           "overlapping subgrid outputs refused");
  }

  // the adjoint over the same three point ranges, every gradient into one
  // buffer per gradient field (point ranges of it)
  {
    const int64_t lo[3] = {0, 5000, 7000}, cnt[3] = {5000, 1, n - 7000};
    std::vector<Dev*> gout;
    for (int f = 0; f < 6; ++f) gout.push_back(new Dev(gc[f] * n));
    tl_domain_bwd doms[3];
    for (int k = 0; k < 3; ++k) {
      auto sub = [&](int f) { return tl_cfield{d[f]->p + lo[k], n}; };
      auto out = [&](int f) { return tl_field{gout[f]->p + lo[k], n}; };
      doms[k] = tl_domain_bwd{cnt[k], sub(0), sub(1), sub(2), sub(4), sub(5), sub(6),
                              out(0), out(1), out(2), out(3), out(4), out(5)};
    }
    tl_batch_plan* plan = nullptr;
    expect(tl_batch_plan_bwd_create(doms, 3, nullptr, &plan) == TL_OK && plan != nullptr,
           "tl_batch_plan_bwd_create");
    if (plan) {
      expect(tl_batch_plan_launch(plan, s) == TL_OK, "adjoint plan launch");
      expect(hipStreamSynchronize(s) == hipSuccess, "adjoint plan sync");
      double worst = 0.0;
      for (int f = 0; f < 6; ++f) {
        const std::vector<double> got = gout[f]->get();
        std::vector<double> a, b;
        for (int c = 0; c < gc[f]; ++c)
          for (int k = 0; k < 3; ++k)
            for (int64_t p = lo[k]; p < lo[k] + cnt[k]; ++p) {
              a.push_back(got[c * n + p]);
              b.push_back(rg[f][c * n + p]);
            }
        const int64_t m = static_cast<int64_t>(a.size()) / gc[f];
        worst = std::fmax(worst, rel_err(a, b, gc[f], m));
      }
      std::printf("adjoint plan rel err %.3e\n", worst);
      expect(worst <= 1e-12, "adjoint plan vs oracle");
      expect(tl_batch_plan_destroy(plan) == TL_OK, "adjoint plan destroy");
    }
    for (auto* x : gout) delete x;
  }

  // argument errors come back before any launch
  expect(tl_dtg_chain(n, tl_cfield{nullptr, n}, cf(1), cf(2), cf(3), cf(4), cf(5),
                      tl_field{dtg.p, n}, s, nullptr) == TL_ERR_NULL, "NULL input");
  expect(tl_dtg_chain(n, cf(0), cf(1), cf(2), cf(3), cf(4), cf(5), tl_field{d[1]->p + 5, n}, s,
                      nullptr) == TL_ERR_ALIAS, "output overlapping an input");
  expect(tl_dtg_chain(n, cf(0), tl_cfield{d[1]->p, n - 1}, cf(2), cf(3), cf(4), cf(5),
                      tl_field{dtg.p, n}, s, nullptr) == TL_ERR_SIZE, "ld < n");
  expect(std::string_view(tl_status_string(TL_ERR_ALIAS)) == "TL_ERR_ALIAS", "status string");
  expect(tl_abi_version() > 0, "abi version");

  (void)hipStreamDestroy(s);
  for (auto* x : d) delete x;
  for (auto* x : gb) delete x;
  for (auto* x : gb2) delete x;
  if (failures) std::printf("c_abi_driver: %d failures\n", failures);
  else std::printf("c_abi_driver: ok\n");
  return failures ? 1 : 0;
}
