// Per-point bodies of the paper's benchmark expressions (Sec. 5.1), device
// code for gfx950, three-dimensional indices.
//
// A non-symmetric rank-r tensor has 3^r components stored row-major over its
// indices (A_ij at i*3+j, A_ijk at (i*3+j)*3+k, ...); a mixed B_i^m is stored
// as B[i*3+m]; K_ij and g_ij are symmetric (s(i,j)).  Inputs are the
// right-hand-side tensors in the order they are written; the output is the
// left-hand side.  Bodies with 81 outputs are streaming bodies (kStream): they
// get a loader ld(field, component) and a storer st(field, component, value) and
// interleave loads, arithmetic and stores in program order, so that only one
// group of outputs is live at a time.
#pragma once

#include "tl_device.hpp"

namespace tl {

constexpr int pow3(int r) { return r == 0 ? 1 : 3 * pow3(r - 1); }

// A_{i..} = B_{i..} for ranks 1..3 (eq:Assign1-3).
template <int R>
struct OpAssign {
  static constexpr int NF_IN = 1, NF_OUT = 1;
  static constexpr int fin[NF_IN] = {pow3(R)};
  static constexpr int fout[NF_OUT] = {pow3(R)};
  static constexpr int NIN = pow3(R), NOUT = pow3(R);
  __device__ static inline void apply(const double* x, double* y) {
#pragma unroll
    for (int c = 0; c < NIN; ++c) y[c] = x[c];
  }
};

// A_i = B_i + C_i (+ D_i (+ E_i)) (eq:Add1-3); M operands.
template <int M>
struct OpAdd {
  static constexpr int NF_IN = M, NF_OUT = 1;
  static constexpr int fin[4] = {3, 3, 3, 3};
  static constexpr int fout[NF_OUT] = {3};
  static constexpr int NIN = 3 * M, NOUT = 3;
  __device__ static inline void apply(const double* x, double* y) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      double s = x[i];
#pragma unroll
      for (int m = 1; m < M; ++m) s += x[3 * m + i];
      y[i] = s;
    }
  }
};

// Outer products A_ij = B_i C_j and A_ijk = B_i C_j D_k (eq:Mult1-2).
template <int M>
struct OpMult {
  static constexpr int NF_IN = M, NF_OUT = 1;
  static constexpr int fin[4] = {3, 3, 3, 3};
  static constexpr int fout[NF_OUT] = {pow3(M)};
  static constexpr int NIN = 3 * M, NOUT = pow3(M);
  __device__ static inline void apply(const double* x, double* y) {
#pragma unroll
    for (int c = 0; c < NOUT; ++c) {
      // base-3 digits of c, most significant first, select B_i, C_j, D_k
      double v = 1.0;
      int rest = c;
#pragma unroll
      for (int m = M - 1; m >= 0; --m) {
        v = m == M - 1 ? x[3 * m + rest % 3] : x[3 * m + rest % 3] * v;
        rest /= 3;
      }
      y[c] = v;
    }
  }
};

// A_ijkl = B_i C_j D_k E_l (eq:Mult3), streaming: the 12 inputs are loaded,
// then each of the 81 outputs is formed and stored in turn.
struct OpMult4 {
  static constexpr bool kStream = true;
  static constexpr int NF_IN = 4, NF_OUT = 1;
  static constexpr int fin[NF_IN] = {3, 3, 3, 3};
  static constexpr int fout[NF_OUT] = {81};
  static constexpr int NIN = 12, NOUT = 81;
  template <class L, class S>
  __device__ static inline void stream(L&& ld, S&& st) {
    double B[3], C[3], D[3], E[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      B[i] = ld(0, i);
      C[i] = ld(1, i);
      D[i] = ld(2, i);
      E[i] = ld(3, i);
    }
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const double bc = B[i] * C[j];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const double bcd = bc * D[k];
#pragma unroll
          for (int l = 0; l < 3; ++l) st(0, ((i * 3 + j) * 3 + k) * 3 + l, bcd * E[l]);
        }
        // Keep the scheduler from forming many outputs ahead of their stores:
        // the kernel is bound by its 81 store streams, and registers held by
        // early products cost occupancy.
        __builtin_amdgcn_sched_barrier(0);
      }
  }
};

// One to three chained contractions (eq:Contract1-3), streaming:
//   A_ijkl = B_i^m E_mjkl:  per (j,k,l), load E_.jkl (3) and store A_.jkl = B E_.jkl;
//   A_ijkl = C_j^n B_i^m E_mnkl:  per (k,l), load the 3x3 E_..kl and store
//     A_..kl = B E_..kl C^T;
//   A_ijkl = D_k^o C_j^n B_i^m E_mnol:  per l, form M_o = B E_..ol C^T for the
//     three o, then store A_..kl = sum_o D_ko M_o for each k.
// Inputs: (B, E), (C, B, E) or (D, C, B, E), as written in the equations.
template <int M>
struct OpContract {
  static constexpr bool kStream = true;
  static constexpr int NF_IN = M + 1, NF_OUT = 1;
  static constexpr int fin[4] = {9, M >= 2 ? 9 : 81, M >= 3 ? 9 : 81, 81};
  static constexpr int fout[NF_OUT] = {81};
  static constexpr int NIN = 9 * M + 81, NOUT = 81;

  static __device__ constexpr int e(int a, int b, int c, int d) {
    return ((a * 3 + b) * 3 + c) * 3 + d;
  }

  // Y = B X C^T for 3x3 matrices (X[m*3+n]).
  __device__ static inline void sandwich(const double* B, const double* X, const double* C,
                                         double* Y) {
    double T[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int n = 0; n < 3; ++n)
        T[i * 3 + n] = B[i * 3 + 0] * X[0 * 3 + n] + B[i * 3 + 1] * X[1 * 3 + n] +
                       B[i * 3 + 2] * X[2 * 3 + n];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j)
        Y[i * 3 + j] = C[j * 3 + 0] * T[i * 3 + 0] + C[j * 3 + 1] * T[i * 3 + 1] +
                       C[j * 3 + 2] * T[i * 3 + 2];
  }

  template <class L, class S>
  __device__ static inline void stream(L&& ld, S&& st) {
    constexpr int fB = M - 1, fE = M;  // field index of B and of E
    double B[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) B[c] = ld(fB, c);
    if constexpr (M == 1) {
#pragma unroll
      for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
          for (int l = 0; l < 3; ++l) {
            const double e0 = ld(fE, e(0, j, k, l)), e1 = ld(fE, e(1, j, k, l)),
                         e2 = ld(fE, e(2, j, k, l));
#pragma unroll
            for (int i = 0; i < 3; ++i)
              st(0, e(i, j, k, l), B[i * 3 + 0] * e0 + B[i * 3 + 1] * e1 + B[i * 3 + 2] * e2);
          }
    } else {
      constexpr int fC = M - 2;
      double C[9];
#pragma unroll
      for (int c = 0; c < 9; ++c) C[c] = ld(fC, c);
      if constexpr (M == 2) {
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
          for (int l = 0; l < 3; ++l) {
            double X[9], Y[9];
#pragma unroll
            for (int m = 0; m < 3; ++m)
#pragma unroll
              for (int n = 0; n < 3; ++n) X[m * 3 + n] = ld(fE, e(m, n, k, l));
            sandwich(B, X, C, Y);
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
              for (int j = 0; j < 3; ++j) st(0, e(i, j, k, l), Y[i * 3 + j]);
          }
      } else {
        double D[9];
#pragma unroll
        for (int c = 0; c < 9; ++c) D[c] = ld(0, c);
#pragma unroll
        for (int l = 0; l < 3; ++l) {
          double Mo[3][9];
#pragma unroll
          for (int o = 0; o < 3; ++o) {
            double X[9];
#pragma unroll
            for (int m = 0; m < 3; ++m)
#pragma unroll
              for (int n = 0; n < 3; ++n) X[m * 3 + n] = ld(fE, e(m, n, o, l));
            sandwich(B, X, C, Mo[o]);
          }
#pragma unroll
          for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int q = 0; q < 9; ++q)
              st(0, e(q / 3, q % 3, k, l),
                 D[k * 3 + 0] * Mo[0][q] + D[k * 3 + 1] * Mo[1][q] + D[k * 3 + 2] * Mo[2][q]);
        }
      }
    }
  }
};

// K_ij = 2 alpha g_ij + beta_i beta_j (eq:Kij).  Inputs alpha, g, beta.
struct OpKij {
  static constexpr int NF_IN = 3, NF_OUT = 1;
  static constexpr int fin[NF_IN] = {1, 6, 3};
  static constexpr int fout[NF_OUT] = {6};
  static constexpr int NIN = 10, NOUT = 6;
  __device__ static inline void apply(const double* x, double* y) {
    const double ta = 2.0 * x[0];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = i; j < 3; ++j) y[sym(i, j)] = ta * x[1 + sym(i, j)] + x[7 + i] * x[7 + j];
  }
};

}  // namespace tl
