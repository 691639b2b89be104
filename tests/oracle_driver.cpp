// Exercises every oracle entry point on small seeded inputs; built with
// AddressSanitizer and UndefinedBehaviorSanitizer by test_oracle_sanitized.py
// (host code only).  Prints one checksum per entry point.
#include <cstdint>
#include <cstdio>
#include <random>
#include <vector>

extern "C" {
void tlo_sym_inverse(int64_t, const double*, double*);
void tlo_christoffel(int64_t, const double*, const double*, double*);
void tlo_christoffel_full(int64_t, const double*, const double*, double*);
void tlo_cov_deriv(int64_t, const double*, const double*, const double*, double*);
void tlo_dtg(int64_t, const double*, const double*, const double*, double*);
void tlo_dtg_chain(int64_t, const double*, const double*, const double*, const double*,
                   const double*, const double*, double*);
void tlo_dtg_chain_jvp(int64_t, const double*, const double*, const double*, const double*,
                       const double*, const double*, const double*, const double*,
                       const double*, const double*, const double*, const double*, double*,
                       double*);
void tlo_dtg_chain_vjp(int64_t, const double*, const double*, const double*, const double*,
                       const double*, const double*, const double*, double*, double*, double*,
                       double*, double*, double*);
int tlo_expr_shape(int, int*, int*, int*);
int tlo_expr(int, int64_t, const double* const*, double*);
}

static std::mt19937_64 rng(12345);
static std::vector<double> field(int ncomp, int64_t n, bool metric = false) {
  std::uniform_real_distribution<double> u(-1.0, 1.0);
  std::vector<double> f(static_cast<size_t>(ncomp * n));
  for (auto& x : f) x = u(rng);
  if (metric)
    for (int64_t p = 0; p < n; ++p) {
      for (int c = 0; c < 6; ++c) f[c * n + p] *= 0.1;
      for (int c : {0, 3, 5}) f[c * n + p] += 1.0;
    }
  return f;
}
static double sum(const std::vector<double>& v) {
  double s = 0.0;
  for (double x : v) s += x;
  return s;
}

int main() {
  const int64_t n = 37;
  auto g = field(6, n, true), dg = field(18, n), b = field(3, n), db = field(9, n),
       K = field(6, n), al = field(1, n), W = field(6, n);
  std::vector<double> gi(6 * n), gam(18 * n), g27(27 * n), nb(9 * n), dtg(6 * n), dot(6 * n);
  tlo_sym_inverse(n, g.data(), gi.data());
  tlo_christoffel(n, gi.data(), dg.data(), gam.data());
  tlo_christoffel_full(n, gi.data(), dg.data(), g27.data());
  tlo_cov_deriv(n, gam.data(), b.data(), db.data(), nb.data());
  tlo_dtg(n, al.data(), K.data(), nb.data(), dtg.data());
  std::printf("steps %.17g %.17g %.17g\n", sum(gi), sum(g27), sum(dtg));
  tlo_dtg_chain(n, g.data(), dg.data(), b.data(), db.data(), K.data(), al.data(), dtg.data());
  tlo_dtg_chain_jvp(n, g.data(), dg.data(), b.data(), db.data(), K.data(), al.data(), g.data(),
                    dg.data(), b.data(), db.data(), K.data(), al.data(), dtg.data(), dot.data());
  std::vector<double> gb(6 * n), dgb(18 * n), bb(3 * n), dbb(9 * n), Kb(6 * n), ab(n);
  tlo_dtg_chain_vjp(n, g.data(), dg.data(), b.data(), db.data(), K.data(), al.data(), W.data(),
                    gb.data(), dgb.data(), bb.data(), dbb.data(), Kb.data(), ab.data());
  tlo_dtg_chain_vjp(n, g.data(), dg.data(), b.data(), db.data(), K.data(), al.data(), W.data(),
                    nullptr, dgb.data(), nullptr, nullptr, nullptr, ab.data());
  std::printf("chain %.17g %.17g %.17g\n", sum(dtg), sum(dot), sum(gb) + sum(dgb));
  for (int id = 0; id < 17; ++id) {
    int nin, ic[4], oc;
    if (tlo_expr_shape(id, &nin, ic, &oc) != 0) return 1;
    std::vector<std::vector<double>> ins;
    std::vector<const double*> ptrs;
    for (int f = 0; f < nin; ++f) ins.push_back(field(ic[f], n));
    for (auto& x : ins) ptrs.push_back(x.data());
    std::vector<double> out(static_cast<size_t>(oc * n), 0.0);
    if (tlo_expr(id, n, ptrs.data(), out.data()) != 0) return 1;
    std::printf("expr %d %.17g\n", id, sum(out));
  }
  return tlo_expr_shape(17, nullptr, nullptr, nullptr) == -1 ? 0 : 1;
}
