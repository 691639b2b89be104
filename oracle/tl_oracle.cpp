// Serial FP64 CPU oracle for the per-grid-point tensor expressions of
// Lewis & Pfeiffer, "Automatic generation of CUDA code performing tensor
// manipulations using C++ expression templates" (arXiv:1804.10120).
//
// TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
// reference that the GPU library is checked against.  It shares no code with
// the GPU path and is only ever called from the tests, from the smoke check and
// from the benchmark's CPU-baseline leg; the product path never calls it.
//
// Every function follows the definition it cites, in the paper's notation and
// operand order, with full index loops over i,j,k,l = 0..2 (the paper's
// 1..3), serially over grid points, in IEEE double (built without fast-math
// and without FP contraction).  Nothing is fused, reassociated or reduced.
//
// Storage conventions (shared with the GPU library's header by value only):
//   a field with C independent components over n points is a contiguous
//   [C][n] array; component c of point p is at ptr[c*n + p].
//   symmetric pair (i,j) -> s(i,j): 00->0 01->1 02->2 11->3 12->4 22->5, the
//     order in which the paper's symmetric loop nests visit the pairs
//     (Sec. 2.4 tensor-index loop; Sec. 3 expression-tree example).
//   dg     [18]: k*6 + s(i,j)  = partial_k g_ij
//   gamma  [18]: i*6 + s(j,k)  = Gamma^i_jk   (symmetric in jk)
//   gamma27[27]: (i*3+j)*3+k   = Gamma^i_jk   (all 27, for symmetry checks)
//   dbeta  [9] : j*3 + i       = partial_j beta_i
//   nabla  [9] : j*3 + i       = nabla_j beta_i
//
// The scalar type is a template parameter so that the same definitions also
// yield exact forward-mode derivatives (dual numbers) and reverse-mode
// gradients (a per-point operation tape); those are the adjoint oracle.

#include <cstdint>
#include <cstddef>
#include <vector>

namespace {

inline int sym(int i, int j) {
  static const int table[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};
  return table[i][j];
}

// ---------------------------------------------------------------------------
// Scalar types.

// Forward-mode dual number: value and directional derivative.
struct Dual {
  double v, d;
  Dual() : v(0.0), d(0.0) {}
  Dual(double x) : v(x), d(0.0) {}
  Dual(double x, double dx) : v(x), d(dx) {}
};
inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(Dual a, Dual b) {
  const double q = a.v / b.v;
  return Dual(q, (a.d - q * b.d) / b.v);
}

// Reverse mode: every operation appends a node holding the indices of its
// (at most two) operands and the partial derivatives with respect to them.
struct Tape {
  std::vector<int> lhs, rhs;
  std::vector<double> dl, dr;
  int push(int a, double da, int b, double db) {
    lhs.push_back(a);
    dl.push_back(da);
    rhs.push_back(b);
    dr.push_back(db);
    return static_cast<int>(lhs.size()) - 1;
  }
  void clear() { lhs.clear(); rhs.clear(); dl.clear(); dr.clear(); }
};
thread_local Tape* g_tape = nullptr;

struct Var {
  double v;
  int id;  // -1: constant, carries no gradient
  Var() : v(0.0), id(-1) {}
  Var(double x) : v(x), id(-1) {}
  static Var leaf(double x) {
    Var r(x);
    r.id = g_tape->push(-1, 0.0, -1, 0.0);
    return r;
  }
};
inline Var make(double v, int a, double da, int b, double db) {
  Var r(v);
  if (a >= 0 || b >= 0) r.id = g_tape->push(a, da, b, db);
  return r;
}
inline Var operator+(Var a, Var b) { return make(a.v + b.v, a.id, 1.0, b.id, 1.0); }
inline Var operator-(Var a, Var b) { return make(a.v - b.v, a.id, 1.0, b.id, -1.0); }
inline Var operator-(Var a) { return make(-a.v, a.id, -1.0, -1, 0.0); }
inline Var operator*(Var a, Var b) { return make(a.v * b.v, a.id, b.v, b.id, a.v); }
inline Var operator/(Var a, Var b) {
  const double q = a.v / b.v;
  return make(q, a.id, 1.0 / b.v, b.id, -q / b.v);
}

// Adjoints of every tape node, given seeds on some nodes.
void sweep(const Tape& t, std::vector<double>& adj) {
  for (int i = static_cast<int>(t.lhs.size()) - 1; i >= 0; --i) {
    const double a = adj[i];
    if (a == 0.0) continue;
    if (t.lhs[i] >= 0) adj[t.lhs[i]] += t.dl[i] * a;
    if (t.rhs[i] >= 0) adj[t.rhs[i]] += t.dr[i] * a;
  }
}

// ---------------------------------------------------------------------------
// Per-point definitions.

// Inverse metric g^ij of the symmetric 3x3 g_ij (Sec. 1, the inverse that
// enters the Christoffel definition; the paper takes it as a given input and
// names no method).  Definition used: Cramer's rule, inverse = adjugate /
// determinant, with the cofactor C_ij = (-1)^(i+j) M_ij written for 3x3 by
// cyclic indices and the determinant expanded along the first row.
template <class T>
void inverse_point(const T g[6], T ginv[6]) {
  T a[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) a[i][j] = g[sym(i, j)];
  T cof[3][3];
  for (int i = 0; i < 3; ++i) {
    const int i1 = (i + 1) % 3, i2 = (i + 2) % 3;
    for (int j = 0; j < 3; ++j) {
      const int j1 = (j + 1) % 3, j2 = (j + 2) % 3;
      cof[i][j] = a[i1][j1] * a[i2][j2] - a[i1][j2] * a[i2][j1];
    }
  }
  T det = a[0][0] * cof[0][0] + a[0][1] * cof[0][1] + a[0][2] * cof[0][2];
  // (g^-1)_ij = adj(g)_ij / det = C_ji / det
  for (int i = 0; i < 3; ++i)
    for (int j = i; j < 3; ++j) ginv[sym(i, j)] = cof[j][i] / det;
}

// Christoffel symbols of the second kind, all 27 (Sec. 1, Christoffel
// definition eq:SpatialChristoffel, and its TLoops form):
//   Gamma^i_jk = 1/2 sum_l g^il (d_k g_jl + d_j g_lk - d_l g_jk).
template <class T>
void christoffel_point(const T ginv[6], const T dg[18], T gam27[27]) {
  auto G = [&](int i, int j) { return ginv[sym(i, j)]; };
  auto D = [&](int k, int i, int j) { return dg[k * 6 + sym(i, j)]; };  // d_k g_ij
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k) {
        T sum(0.0);
        for (int l = 0; l < 3; ++l)
          sum = sum + G(i, l) * ((D(k, j, l) + D(j, l, k)) - D(l, j, k));
        gam27[(i * 3 + j) * 3 + k] = T(0.5) * sum;
      }
}

// Covariant derivative of the shift covector (Sec. 1, footnote to the
// schematic dtg listing):  nabla_j beta_i = d_j beta_i - Gamma^k_ij beta_k.
template <class T>
void cov_deriv_point(const T gam27[27], const T beta[3], const T dbeta[9], T nb[9]) {
  for (int j = 0; j < 3; ++j)
    for (int i = 0; i < 3; ++i) {
      T sum(0.0);
      for (int k = 0; k < 3; ++k) sum = sum + gam27[(k * 3 + i) * 3 + j] * beta[k];
      nb[j * 3 + i] = dbeta[j * 3 + i] - sum;
    }
}

// Metric evolution (Sec. 1, eq:dtg_ij and the schematic/TLoops listings):
//   d_t g_ij = -2 alpha K_ij + nabla_i beta_j + nabla_j beta_i,
// evaluated for i >= j, the member the paper's loops for the Sym<0,1>
// left-hand side visit (Sec. 2.4: the first index starts at the second).
template <class T>
void dtg_point(const T& alpha, const T K[6], const T nb[9], T dtg[6]) {
  for (int j = 0; j < 3; ++j)
    for (int i = j; i < 3; ++i)
      dtg[sym(i, j)] = T(-2.0) * alpha * K[sym(i, j)] + nb[i * 3 + j] + nb[j * 3 + i];
}

// The chain, step by step: inverse, Christoffel, covariant derivative, dtg.
template <class T>
void chain_point(const T g[6], const T dg[18], const T beta[3], const T dbeta[9], const T K[6],
                 const T& alpha, T dtg[6]) {
  T ginv[6], gam27[27], nb[9];
  inverse_point(g, ginv);
  christoffel_point(ginv, dg, gam27);
  cov_deriv_point(gam27, beta, dbeta, nb);
  dtg_point(alpha, K, nb, dtg);
}

// Field access helpers for contiguous [C][n] arrays.
template <class T>
inline void gather(const double* f, int64_t n, int64_t p, int ncomp, T* out) {
  for (int c = 0; c < ncomp; ++c) out[c] = T(f[c * n + p]);
}
inline void scatter(double* f, int64_t n, int64_t p, int ncomp, const double* in) {
  for (int c = 0; c < ncomp; ++c) f[c * n + p] = in[c];
}

}  // namespace

extern "C" {

int tlo_abi_version(void) { return 1; }

void tlo_sym_inverse(int64_t n, const double* g, double* ginv) {
  for (int64_t p = 0; p < n; ++p) {
    double a[6], r[6];
    gather(g, n, p, 6, a);
    inverse_point(a, r);
    scatter(ginv, n, p, 6, r);
  }
}

void tlo_christoffel_full(int64_t n, const double* ginv, const double* dg, double* gamma27) {
  for (int64_t p = 0; p < n; ++p) {
    double G[6], D[18], r[27];
    gather(ginv, n, p, 6, G);
    gather(dg, n, p, 18, D);
    christoffel_point(G, D, r);
    scatter(gamma27, n, p, 27, r);
  }
}

void tlo_christoffel(int64_t n, const double* ginv, const double* dg, double* gamma) {
  for (int64_t p = 0; p < n; ++p) {
    double G[6], D[18], r[27], out[18];
    gather(ginv, n, p, 6, G);
    gather(dg, n, p, 18, D);
    christoffel_point(G, D, r);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        for (int k = j; k < 3; ++k) out[i * 6 + sym(j, k)] = r[(i * 3 + j) * 3 + k];
    scatter(gamma, n, p, 18, out);
  }
}

void tlo_cov_deriv(int64_t n, const double* gamma, const double* beta, const double* dbeta,
                   double* nabla) {
  for (int64_t p = 0; p < n; ++p) {
    double Gs[18], g27[27], b[3], db[9], r[9];
    gather(gamma, n, p, 18, Gs);
    gather(beta, n, p, 3, b);
    gather(dbeta, n, p, 9, db);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        for (int k = 0; k < 3; ++k) g27[(i * 3 + j) * 3 + k] = Gs[i * 6 + sym(j, k)];
    cov_deriv_point(g27, b, db, r);
    scatter(nabla, n, p, 9, r);
  }
}

void tlo_dtg(int64_t n, const double* alpha, const double* K, const double* nabla, double* dtg) {
  for (int64_t p = 0; p < n; ++p) {
    double k6[6], nb[9], r[6];
    gather(K, n, p, 6, k6);
    gather(nabla, n, p, 9, nb);
    dtg_point(alpha[p], k6, nb, r);
    scatter(dtg, n, p, 6, r);
  }
}

void tlo_dtg_chain(int64_t n, const double* g, const double* dg, const double* beta,
                   const double* dbeta, const double* K, const double* alpha, double* dtg) {
  for (int64_t p = 0; p < n; ++p) {
    double a[6], D[18], b[3], db[9], k6[6], r[6];
    gather(g, n, p, 6, a);
    gather(dg, n, p, 18, D);
    gather(beta, n, p, 3, b);
    gather(dbeta, n, p, 9, db);
    gather(K, n, p, 6, k6);
    chain_point(a, D, b, db, k6, alpha[p], r);
    scatter(dtg, n, p, 6, r);
  }
}

// Forward-mode derivative of the chain: dtg and its directional derivative
// along the tangent fields (t_g, ..., t_alpha), exact up to rounding.
void tlo_dtg_chain_jvp(int64_t n, const double* g, const double* dg, const double* beta,
                       const double* dbeta, const double* K, const double* alpha,
                       const double* tg, const double* tdg, const double* tbeta,
                       const double* tdbeta, const double* tK, const double* talpha, double* dtg,
                       double* dtg_dot) {
  for (int64_t p = 0; p < n; ++p) {
    Dual a[6], D[18], b[3], db[9], k6[6], r[6];
    for (int c = 0; c < 6; ++c) a[c] = Dual(g[c * n + p], tg[c * n + p]);
    for (int c = 0; c < 18; ++c) D[c] = Dual(dg[c * n + p], tdg[c * n + p]);
    for (int c = 0; c < 3; ++c) b[c] = Dual(beta[c * n + p], tbeta[c * n + p]);
    for (int c = 0; c < 9; ++c) db[c] = Dual(dbeta[c * n + p], tdbeta[c * n + p]);
    for (int c = 0; c < 6; ++c) k6[c] = Dual(K[c * n + p], tK[c * n + p]);
    const Dual al(alpha[p], talpha[p]);
    chain_point(a, D, b, db, k6, al, r);
    for (int c = 0; c < 6; ++c) {
      dtg[c * n + p] = r[c].v;
      dtg_dot[c * n + p] = r[c].d;
    }
  }
}

// Reverse-mode gradient of L = sum_p sum_s W_s(p) dtg_s(p) with respect to
// every stored input component (an off-diagonal stored slot of g, dg or K
// receives the sum of its (i,j) and (j,i) partials, because both read the same
// stored value).  Any output pointer may be NULL to skip that gradient.
void tlo_dtg_chain_vjp(int64_t n, const double* g, const double* dg, const double* beta,
                       const double* dbeta, const double* K, const double* alpha, const double* W,
                       double* g_bar, double* dg_bar, double* beta_bar, double* dbeta_bar,
                       double* K_bar, double* alpha_bar) {
  Tape tape;
  g_tape = &tape;
  std::vector<double> adj;
  for (int64_t p = 0; p < n; ++p) {
    tape.clear();
    Var a[6], D[18], b[3], db[9], k6[6], r[6];
    for (int c = 0; c < 6; ++c) a[c] = Var::leaf(g[c * n + p]);
    for (int c = 0; c < 18; ++c) D[c] = Var::leaf(dg[c * n + p]);
    for (int c = 0; c < 3; ++c) b[c] = Var::leaf(beta[c * n + p]);
    for (int c = 0; c < 9; ++c) db[c] = Var::leaf(dbeta[c * n + p]);
    for (int c = 0; c < 6; ++c) k6[c] = Var::leaf(K[c * n + p]);
    const Var al = Var::leaf(alpha[p]);
    chain_point(a, D, b, db, k6, al, r);
    adj.assign(tape.lhs.size(), 0.0);
    for (int c = 0; c < 6; ++c)
      if (r[c].id >= 0) adj[r[c].id] += W[c * n + p];
    sweep(tape, adj);
    auto grad = [&](const Var& v) { return v.id >= 0 ? adj[v.id] : 0.0; };
    if (g_bar)
      for (int c = 0; c < 6; ++c) g_bar[c * n + p] = grad(a[c]);
    if (dg_bar)
      for (int c = 0; c < 18; ++c) dg_bar[c * n + p] = grad(D[c]);
    if (beta_bar)
      for (int c = 0; c < 3; ++c) beta_bar[c * n + p] = grad(b[c]);
    if (dbeta_bar)
      for (int c = 0; c < 9; ++c) dbeta_bar[c * n + p] = grad(db[c]);
    if (K_bar)
      for (int c = 0; c < 6; ++c) K_bar[c * n + p] = grad(k6[c]);
    if (alpha_bar) alpha_bar[p] = grad(al);
  }
  g_tape = nullptr;
}

// ---------------------------------------------------------------------------
// The benchmark expressions of Sec. 5.1 (eq:Assign1-3, eq:Add1-3,
// eq:Mult1-3, eq:Contract1-3, eq:Kij), with three-dimensional indices.  A
// non-symmetric tensor of rank r has 3^r components stored row-major over its
// indices (A_ij at i*3+j, A_ijk at (i*3+j)*3+k, ...); a mixed B_i^m is stored
// as B[i*3+m]; K_ij and g_ij are symmetric (6 components, s(i,j)); alpha is a
// scalar field.  Inputs are the right-hand-side tensors in the order they are
// written in the equation; the output is the left-hand side.
//
//   id  expression                              inputs (components)     out
//    0  A_i = B_i                               3                        3
//    1  A_ij = B_ij                             9                        9
//    2  A_ijk = B_ijk                           27                       27
//    3  A_i = B_i + C_i                         3 3                      3
//    4  A_i = B_i + C_i + D_i                   3 3 3                    3
//    5  A_i = B_i + C_i + D_i + E_i             3 3 3 3                  3
//    6  A_ij = B_i C_j                          3 3                      9
//    7  A_ijk = B_i C_j D_k                     3 3 3                    27
//    8  A_ijkl = B_i C_j D_k E_l                3 3 3 3                  81
//    9  A_ijkl = B_i^m E_mjkl                   9 81                     81
//   10  A_ijkl = C_j^n B_i^m E_mnkl             9 9 81                   81
//   11  A_ijkl = D_k^o C_j^n B_i^m E_mnol       9 9 9 81                 81
//   12  K_ij = 2 alpha g_ij + beta_i beta_j     1 6 3                    6
//
// And, with four-dimensional (spacetime) indices a,b,c = 0..3 and the
// symmetric dimension-4 pair order of the same kind (00 01 02 03 11 12 13 22 23
// 33), the examples of Sec. 4 and the spacetime split of Sec. 2.2:
//   13  C_(ab) = sum_c A_ac B_cb  (symmetric LHS)    16 16     10
//   14  D_(i0) = sum_c E_(i+1)c F_c0, i = 0..2       16 16     10 (3 written)
//   15  g_ij = psi_(i+1)(j+1)                         10        6
//   16  beta_i = psi_(i+1)0                           10        3
// For a symmetric left-hand side with both slots free, each stored pair is
// evaluated at the member whose first index is >= the second: the paper's
// loops for a Sym<0,1> left-hand side start the first index at the value of
// the second (the tensor-index loop of Sec. 2.4, and the generated C loop and
// CUDA kernel of the rank-2 contraction example in Sec. 4).  For a right-hand
// side that is not symmetric this decides which of C_ab and C_ba is stored.
namespace {

inline int sym4(int a, int b) {
  static const int table[4][4] = {{0, 1, 2, 3}, {1, 4, 5, 6}, {2, 5, 7, 8}, {3, 6, 8, 9}};
  return table[a][b];
}

int ipow3(int r) { return r == 0 ? 1 : 3 * ipow3(r - 1); }

void expr_point(int id, const std::vector<const double*>& in, double* out) {
  switch (id) {
    case 0:
    case 1:
    case 2: {
      const int m = ipow3(id + 1);
      for (int c = 0; c < m; ++c) out[c] = in[0][c];
      break;
    }
    case 3:
      for (int i = 0; i < 3; ++i) out[i] = in[0][i] + in[1][i];
      break;
    case 4:
      for (int i = 0; i < 3; ++i) out[i] = in[0][i] + in[1][i] + in[2][i];
      break;
    case 5:
      for (int i = 0; i < 3; ++i) out[i] = in[0][i] + in[1][i] + in[2][i] + in[3][i];
      break;
    case 6:
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) out[i * 3 + j] = in[0][i] * in[1][j];
      break;
    case 7:
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
          for (int k = 0; k < 3; ++k) out[(i * 3 + j) * 3 + k] = in[0][i] * in[1][j] * in[2][k];
      break;
    case 8:
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
          for (int k = 0; k < 3; ++k)
            for (int l = 0; l < 3; ++l)
              out[((i * 3 + j) * 3 + k) * 3 + l] = in[0][i] * in[1][j] * in[2][k] * in[3][l];
      break;
    case 9: {  // B = in[0], E = in[1]
      const double *B = in[0], *E = in[1];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
          for (int k = 0; k < 3; ++k)
            for (int l = 0; l < 3; ++l) {
              double sum = 0.0;
              for (int m = 0; m < 3; ++m) sum += B[i * 3 + m] * E[((m * 3 + j) * 3 + k) * 3 + l];
              out[((i * 3 + j) * 3 + k) * 3 + l] = sum;
            }
      break;
    }
    case 10: {  // C = in[0], B = in[1], E = in[2]
      const double *C = in[0], *B = in[1], *E = in[2];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
          for (int k = 0; k < 3; ++k)
            for (int l = 0; l < 3; ++l) {
              double sum = 0.0;
              for (int n = 0; n < 3; ++n)
                for (int m = 0; m < 3; ++m)
                  sum += C[j * 3 + n] * B[i * 3 + m] * E[((m * 3 + n) * 3 + k) * 3 + l];
              out[((i * 3 + j) * 3 + k) * 3 + l] = sum;
            }
      break;
    }
    case 11: {  // D = in[0], C = in[1], B = in[2], E = in[3]
      const double *D = in[0], *C = in[1], *B = in[2], *E = in[3];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
          for (int k = 0; k < 3; ++k)
            for (int l = 0; l < 3; ++l) {
              double sum = 0.0;
              for (int o = 0; o < 3; ++o)
                for (int n = 0; n < 3; ++n)
                  for (int m = 0; m < 3; ++m)
                    sum += D[k * 3 + o] * C[j * 3 + n] * B[i * 3 + m] *
                           E[((m * 3 + n) * 3 + o) * 3 + l];
              out[((i * 3 + j) * 3 + k) * 3 + l] = sum;
            }
      break;
    }
    case 12: {  // alpha = in[0], g = in[1], beta = in[2]
      const double alpha = in[0][0];
      for (int j = 0; j < 3; ++j)
        for (int i = j; i < 3; ++i)
          out[sym(i, j)] = 2.0 * alpha * in[1][sym(i, j)] + in[2][i] * in[2][j];
      break;
    }
    case 13: {  // A = in[0], B = in[1], both 4x4 row-major; evaluated for a >= b
      for (int b = 0; b < 4; ++b)
        for (int a = b; a < 4; ++a) {
          double sum = 0.0;
          for (int c = 0; c < 4; ++c) sum += in[0][a * 4 + c] * in[1][c * 4 + b];
          out[sym4(a, b)] = sum;
        }
      break;
    }
    case 14: {  // E = in[0], F = in[1], both 4x4 row-major; only D_(i0) is written
      for (int i = 0; i < 3; ++i) {
        double sum = 0.0;
        for (int c = 0; c < 4; ++c) sum += in[0][(i + 1) * 4 + c] * in[1][c * 4 + 0];
        out[sym4(i, 0)] = sum;
      }
      break;
    }
    case 15:
      for (int j = 0; j < 3; ++j)
        for (int i = j; i < 3; ++i) out[sym(i, j)] = in[0][sym4(i + 1, j + 1)];
      break;
    case 16:
      for (int i = 0; i < 3; ++i) out[i] = in[0][sym4(i + 1, 0)];
      break;
    default:
      break;
  }
}

const int kExprIn[17][4] = {{3}, {9}, {27}, {3, 3}, {3, 3, 3}, {3, 3, 3, 3}, {3, 3}, {3, 3, 3},
                            {3, 3, 3, 3}, {9, 81}, {9, 9, 81}, {9, 9, 9, 81}, {1, 6, 3},
                            {16, 16}, {16, 16}, {10}, {10}};
const int kExprOut[17] = {3, 9, 27, 3, 3, 3, 9, 27, 81, 81, 81, 81, 6, 10, 10, 6, 3};

}  // namespace

// Shape of expression `id`: number of inputs, their component counts and the
// output's; returns 0, or -1 for an unknown id.
int tlo_expr_shape(int id, int* nin, int* in_ncomp, int* out_ncomp) {
  if (id < 0 || id > 16) return -1;
  int k = 0;
  while (k < 4 && kExprIn[id][k] > 0) {
    in_ncomp[k] = kExprIn[id][k];
    ++k;
  }
  *nin = k;
  *out_ncomp = kExprOut[id];
  return 0;
}

// Expression `id` over n points; in[] are contiguous [C][n] inputs in the
// order of the table above, out a contiguous [C][n] output.
int tlo_expr(int id, int64_t n, const double* const* in, double* out) {
  int nin, ic[4], oc;
  if (tlo_expr_shape(id, &nin, ic, &oc) != 0) return -1;
  std::vector<std::vector<double>> x(nin);
  for (int f = 0; f < nin; ++f) x[f].resize(ic[f]);
  std::vector<const double*> xp(nin);
  std::vector<double> y(oc);
  for (int64_t p = 0; p < n; ++p) {
    for (int f = 0; f < nin; ++f) {
      for (int c = 0; c < ic[f]; ++c) x[f][c] = in[f][c * n + p];
      xp[f] = x[f].data();
    }
    for (int c = 0; c < oc; ++c) y[c] = out[c * n + p];  // components not written stay
    expr_point(id, xp, y.data());
    for (int c = 0; c < oc; ++c) out[c * n + p] = y[c];
  }
  return 0;
}

}  // extern "C"
