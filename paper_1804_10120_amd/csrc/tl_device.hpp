// Per-grid-point bodies of the tensor expressions (device code, gfx950).
//
// Every body maps the components of one grid point, gathered into registers,
// to the output components of that point.  The kernel templates (tl_stream.hpp)
// load and store the components (component-major fields, one coalesced stream
// per component) and call these bodies; all index arithmetic below is on
// compile-time constants, so after unrolling every tensor lives in registers.
//
// Component orders are those of include/tl.h: symmetric pair s(i,j) in the
// order 00 01 02 11 12 22; dg[k*6+s(i,j)] = d_k g_ij; gamma[i*6+s(j,k)] =
// Gamma^i_jk; dbeta[j*3+i] = d_j beta_i; nabla[j*3+i] = nabla_j beta_i.
#pragma once

#include <cstdint>

namespace tl {

__host__ __device__ constexpr int sym(int i, int j) {
  return i <= j ? (i == 0 ? j : (i == 1 ? 2 + j : 5)) : (j == 0 ? i : (j == 1 ? 2 + i : 5));
}

// Cofactors of the symmetric g (stored order) and the determinant; the
// inverse is cof * (1/det).  cof is symmetric, stored in the same order.
__device__ inline void cofactors(const double* g, double* cof, double& det) {
  const double g00 = g[0], g01 = g[1], g02 = g[2], g11 = g[3], g12 = g[4], g22 = g[5];
  cof[0] = g11 * g22 - g12 * g12;
  cof[1] = g02 * g12 - g01 * g22;
  cof[2] = g01 * g12 - g02 * g11;
  cof[3] = g00 * g22 - g02 * g02;
  cof[4] = g01 * g02 - g00 * g12;
  cof[5] = g00 * g11 - g01 * g01;
  det = g00 * cof[0] + g01 * cof[1] + g02 * cof[2];
}

// ---------------------------------------------------------------- inverse
// g^ij of the symmetric 3x3 g_ij (the inverse metric of the Christoffel
// definition, Sec. 1, eq:SpatialChristoffel): adjugate times one IEEE
// reciprocal of the determinant.
struct OpSymInverse {
  static constexpr int NF_IN = 1, NF_OUT = 1;
  static constexpr int fin[NF_IN] = {6};
  static constexpr int fout[NF_OUT] = {6};
  static constexpr int NIN = 6, NOUT = 6;
  __device__ static inline void apply(const double* x, double* y) {
    double cof[6], det;
    cofactors(x, cof, det);
    const double r = 1.0 / det;
#pragma unroll
    for (int s = 0; s < 6; ++s) y[s] = cof[s] * r;
  }
};

// ---------------------------------------------------------------- Christoffel
// Gamma^i_jk (Sec. 1, eq:SpatialChristoffel) = sum_l g^il Gamma_ljk with the
// first-kind symbols
// Gamma_ljk = 1/2 (d_k g_jl + d_j g_lk - d_l g_jk) (each needed once per l and
// pair jk, so 18 of them, then 54 multiply-adds to raise the index).
struct OpChristoffel {
  static constexpr int NF_IN = 2, NF_OUT = 1;
  static constexpr int fin[NF_IN] = {6, 18};
  static constexpr int fout[NF_OUT] = {18};
  static constexpr int NIN = 24, NOUT = 18;
  __device__ static inline void apply(const double* x, double* y) {
    const double* G = x;       // g^ij
    const double* D = x + 6;   // d_k g_ij
    double first[3][6];
#pragma unroll
    for (int l = 0; l < 3; ++l)
#pragma unroll
      for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int k = j; k < 3; ++k)
          first[l][sym(j, k)] =
              0.5 * (D[k * 6 + sym(j, l)] + D[j * 6 + sym(l, k)] - D[l * 6 + sym(j, k)]);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int s = 0; s < 6; ++s)
        y[i * 6 + s] = G[sym(i, 0)] * first[0][s] + G[sym(i, 1)] * first[1][s] +
                       G[sym(i, 2)] * first[2][s];
  }
};

// ---------------------------------------------------------------- nabla beta
// nabla_j beta_i = d_j beta_i - Gamma^k_ij beta_k (Sec. 1, the footnote to the
// schematic listing of eq:dtg_ij).
struct OpCovDeriv {
  static constexpr int NF_IN = 3, NF_OUT = 1;
  static constexpr int fin[NF_IN] = {18, 3, 9};
  static constexpr int fout[NF_OUT] = {9};
  static constexpr int NIN = 30, NOUT = 9;
  __device__ static inline void apply(const double* x, double* y) {
    const double* Gam = x;
    const double* b = x + 18;
    const double* db = x + 21;
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const int s = sym(i, j);
        y[j * 3 + i] = db[j * 3 + i] - (Gam[s] * b[0] + Gam[6 + s] * b[1] + Gam[12 + s] * b[2]);
      }
  }
};

// ---------------------------------------------------------------- d_t g
// d_t g_ij = -2 alpha K_ij + nabla_i beta_j + nabla_j beta_i (Sec. 1, eq:dtg_ij).
struct OpDtg {
  static constexpr int NF_IN = 3, NF_OUT = 1;
  static constexpr int fin[NF_IN] = {1, 6, 9};
  static constexpr int fout[NF_OUT] = {6};
  static constexpr int NIN = 16, NOUT = 6;
  __device__ static inline void apply(const double* x, double* y) {
    const double m2a = -2.0 * x[0];
    const double* K = x + 1;
    const double* nb = x + 7;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = i; j < 3; ++j) y[sym(i, j)] = m2a * K[sym(i, j)] + (nb[i * 3 + j] + nb[j * 3 + i]);
  }
};

// ---------------------------------------------------------------- fused chain
// Reduced form of the chain (eq:dtg_ij with eq:SpatialChristoffel substituted,
// Sec. 1).  With b^l = g^lk beta_k,
//   Gamma^k_ij beta_k = 1/2 b^l (d_j g_il + d_i g_lj - d_l g_ij),
// so with A[k][i] = sum_l b^l d_k g_il and B_ij = sum_l b^l d_l g_ij
//   d_t g_ij = -2 alpha K_ij + d_i beta_j + d_j beta_i - (A[j][i] + A[i][j] - B_ij).
// g^ij itself is never formed: b = adj(g) beta / det.
struct OpChain {
  static constexpr int NF_IN = 6, NF_OUT = 1;
  static constexpr int fin[NF_IN] = {6, 18, 3, 9, 6, 1};
  static constexpr int fout[NF_OUT] = {6};
  static constexpr int NIN = 43, NOUT = 6;
  __device__ static inline void apply(const double* x, double* y) {
    const double* g = x;
    const double* D = x + 6;
    const double* beta = x + 24;
    const double* db = x + 27;
    const double* K = x + 36;
    const double alpha = x[42];
    double cof[6], det;
    cofactors(g, cof, det);
    const double r = 1.0 / det;
    double b[3];
#pragma unroll
    for (int l = 0; l < 3; ++l)
      b[l] = (cof[sym(l, 0)] * beta[0] + cof[sym(l, 1)] * beta[1] + cof[sym(l, 2)] * beta[2]) * r;
    double A[3][3], B[6];
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int i = 0; i < 3; ++i)
        A[k][i] = b[0] * D[k * 6 + sym(i, 0)] + b[1] * D[k * 6 + sym(i, 1)] +
                  b[2] * D[k * 6 + sym(i, 2)];
#pragma unroll
    for (int s = 0; s < 6; ++s) B[s] = b[0] * D[s] + b[1] * D[6 + s] + b[2] * D[12 + s];
    const double m2a = -2.0 * alpha;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = i; j < 3; ++j) {
        const int s = sym(i, j);
        y[s] = m2a * K[s] + (db[i * 3 + j] + db[j * 3 + i]) - ((A[j][i] + A[i][j]) - B[s]);
      }
  }
};

// ---------------------------------------------------------------- adjoint
// Vector-Jacobian product of OpChain for w = dL/d(d_t g), gradients with
// respect to the stored components.  With b = g^-1 beta and
// F_l,ij = d_j g_il + d_i g_lj - d_l g_ij (so d_t g_ij = ... - b^l F_l,ij):
//   K_bar_ij     = -2 alpha w_ij
//   alpha_bar    = -2 sum_s w_s K_s
//   dbeta_bar    : d_j beta_i enters d_t g_s(i,j) once for i != j and twice for
//                  i == j, so dbeta_bar[j][i] = w_s(i,j) (times 2 on the diagonal)
//   b_bar^l      = -sum_s w_s F_l,s
//   beta_bar     = g^-1 b_bar
//   g_bar(full)  = -g^-1 b_bar beta^T g^-1 = -beta_bar b^T, so a stored slot
//                  gets -(beta_bar_i b^j + beta_bar_j b^i) off the diagonal and
//                  -beta_bar_i b^i on it
//   dg_bar       : d_k g_ab appears in F with coefficient -w_s b^l at the
//                  three places F names; scattered below.
// Inputs: g 6, dg 18, beta 3, K 6, alpha 1, w 6.  Outputs (in this order):
// g_bar 6, dg_bar 18, beta_bar 3, dbeta_bar 9, K_bar 6, alpha_bar 1.
struct OpChainBwd {
  static constexpr int NF_IN = 6, NF_OUT = 6;
  static constexpr int fin[NF_IN] = {6, 18, 3, 6, 1, 6};
  static constexpr int fout[NF_OUT] = {6, 18, 3, 9, 6, 1};
  static constexpr int NIN = 40, NOUT = 43;

  // Everything that does not need d g: b = g^-1 beta (kept as cofactors, 1/det
  // and b for phase2) and the gradients with respect to K, alpha, d beta and
  // d g, which depend on w, alpha, K and b only.
  __device__ static inline void phase1(const double* g, const double* beta, const double* K,
                                       double alpha, const double* w, double* cof, double& r,
                                       double* b, double* dg_bar, double* dbeta_bar,
                                       double* K_bar, double* alpha_bar) {
    double det;
    cofactors(g, cof, det);
    r = 1.0 / det;
#pragma unroll
    for (int l = 0; l < 3; ++l)
      b[l] = (cof[sym(l, 0)] * beta[0] + cof[sym(l, 1)] * beta[1] + cof[sym(l, 2)] * beta[2]) * r;

    const double m2a = -2.0 * alpha;
    double ab = 0.0;
#pragma unroll
    for (int s = 0; s < 6; ++s) {
      K_bar[s] = m2a * w[s];
      ab += w[s] * K[s];
    }
    alpha_bar[0] = -2.0 * ab;
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int i = 0; i < 3; ++i) dbeta_bar[j * 3 + i] = (i == j ? 2.0 : 1.0) * w[sym(i, j)];

    // dg_bar: for every stored pair (i,j) and every l, c = -w_ij b^l is added
    // to d_j g_il and d_i g_lj and subtracted from d_l g_ij.
#pragma unroll
    for (int q = 0; q < 18; ++q) dg_bar[q] = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = i; j < 3; ++j) {
        const int s = sym(i, j);
#pragma unroll
        for (int l = 0; l < 3; ++l) {
          const double c = -w[s] * b[l];
          dg_bar[j * 6 + sym(i, l)] += c;
          dg_bar[i * 6 + sym(l, j)] += c;
          dg_bar[l * 6 + s] -= c;
        }
      }
  }

  // The gradients that need d g: b_bar^l = -sum_s w_s F_l,s, beta_bar =
  // g^-1 b_bar and g_bar = -beta_bar b^T on the stored slots.
  __device__ static inline void phase2(const double* D, const double* w, const double* cof,
                                       double r, const double* b, double* g_bar,
                                       double* beta_bar) {
    double bb[3];
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      double acc = 0.0;
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = i; j < 3; ++j) {
          const int s = sym(i, j);
          acc += w[s] * ((D[j * 6 + sym(i, l)] + D[i * 6 + sym(l, j)]) - D[l * 6 + s]);
        }
      bb[l] = -acc;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k)
      beta_bar[k] = (cof[sym(k, 0)] * bb[0] + cof[sym(k, 1)] * bb[1] + cof[sym(k, 2)] * bb[2]) * r;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = i; j < 3; ++j)
        g_bar[sym(i, j)] =
            i == j ? -(beta_bar[i] * b[i]) : -(beta_bar[i] * b[j] + beta_bar[j] * b[i]);
  }

  __device__ static inline void apply(const double* x, double* y) {
    double cof[6], r, b[3];
    phase1(x, x + 24, x + 27, x[33], x + 34, cof, r, b, y + 6, y + 27, y + 36, y + 42);
    phase2(x + 6, x + 34, cof, r, b, y, y + 24);
  }
};

// ---------------------------------------------------------------- value and gradient
// d_t g and its vector-Jacobian product for a cotangent w that is known when
// the chain is evaluated (a loss linear in d_t g, such as sum_s w_s d_t g_s):
// OpChain and OpChainBwd on one read of the shared inputs.  Inputs: g 6, dg 18,
// beta 3, dbeta 9, K 6, alpha 1, w 6.  Outputs: d_t g 6, then the six
// gradients of OpChainBwd in its order.
struct OpChainFwdBwd {
  static constexpr int NF_IN = 7, NF_OUT = 7;
  static constexpr int fin[NF_IN] = {6, 18, 3, 9, 6, 1, 6};
  static constexpr int fout[NF_OUT] = {6, 6, 18, 3, 9, 6, 1};
  static constexpr int NIN = 49, NOUT = 49;
  __device__ static inline void apply(const double* x, double* y) {
    OpChain::apply(x, y);
    double cof[6], r, b[3];
    OpChainBwd::phase1(x, x + 24, x + 36, x[42], x + 43, cof, r, b, y + 12, y + 33, y + 42,
                       y + 48);
    OpChainBwd::phase2(x + 6, x + 43, cof, r, b, y + 6, y + 30);
  }
};

// ---------------------------------------------------------------- twin
// Bandwidth twin of a row: reads NI component streams and writes NO, with no
// arithmetic beyond a sum (each output is the sum of the inputs plus its own
// index), so it measures the memory ceiling of that access shape.
template <int NI, int NO>
struct OpTwin {
  static constexpr int NF_IN = 1, NF_OUT = 1;
  static constexpr int fin[NF_IN] = {NI};
  static constexpr int fout[NF_OUT] = {NO};
  static constexpr int NIN = NI, NOUT = NO;
  __device__ static inline void apply(const double* x, double* y) {
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < NI; ++i) s += x[i];
#pragma unroll
    for (int o = 0; o < NO; ++o) y[o] = s + static_cast<double>(o);
  }
};

}  // namespace tl
