// Generated from index notation by paper_1804_10120_amd/codegen (regenerate
// with `python -m paper_1804_10120_amd.codegen`, do not edit by hand).
// Streaming per-point bodies for gfx950 and their C-ABI entry points; see
// include/tl_generated.h for the expressions.
#include <hip/hip_runtime.h>

#include "../../../include/tl_generated.h"
#include "../tl_internal.hpp"
#include "../tl_stream.hpp"

namespace tl {

// christoffel: Christoffel symbols from g^ij and d_k g_ij (Sec. 1, eq:SpatialChristoffel)
struct Gen_christoffel {
  static constexpr bool kStream = true;
  static constexpr int NF_IN = 2, NF_OUT = 1;
  static constexpr int fin[NF_IN] = {6, 18};
  static constexpr int fout[NF_OUT] = {18};
  static constexpr int NIN = 24, NOUT = 18;
  template <class L, class S>
  __device__ static inline void stream(L&& ld, S&& st) {
    const double x0_0 = ld(0, 0);
    const double x0_1 = ld(0, 1);
    const double x0_2 = ld(0, 2);
    const double x0_3 = ld(0, 3);
    const double x0_4 = ld(0, 4);
    const double x0_5 = ld(0, 5);
    const double x1_0 = ld(1, 0);
    const double x1_1 = ld(1, 1);
    const double x1_2 = ld(1, 2);
    const double x1_3 = ld(1, 3);
    const double x1_4 = ld(1, 4);
    const double x1_5 = ld(1, 5);
    const double x1_6 = ld(1, 6);
    const double x1_7 = ld(1, 7);
    const double x1_8 = ld(1, 8);
    const double x1_9 = ld(1, 9);
    const double x1_10 = ld(1, 10);
    const double x1_11 = ld(1, 11);
    const double x1_12 = ld(1, 12);
    const double x1_13 = ld(1, 13);
    const double x1_14 = ld(1, 14);
    const double x1_15 = ld(1, 15);
    const double x1_16 = ld(1, 16);
    const double x1_17 = ld(1, 17);
    // Gamma(i,j,k) = (0.5 * Sum(l, (Invg(i,l) * ((dg(k,j,l) + dg(j,l,k)) - dg(l,j,k)))))
    double o0_0 = (0.5 * ((x0_0 * ((x1_0 + x1_0) - x1_0)) + (x0_1 * ((x1_1 + x1_1) - x1_6)) + (x0_2 * ((x1_2 + x1_2) - x1_12))));
    st(0, 0, o0_0);
    double o0_6 = (0.5 * ((x0_1 * ((x1_0 + x1_0) - x1_0)) + (x0_3 * ((x1_1 + x1_1) - x1_6)) + (x0_4 * ((x1_2 + x1_2) - x1_12))));
    st(0, 6, o0_6);
    double o0_12 = (0.5 * ((x0_2 * ((x1_0 + x1_0) - x1_0)) + (x0_4 * ((x1_1 + x1_1) - x1_6)) + (x0_5 * ((x1_2 + x1_2) - x1_12))));
    st(0, 12, o0_12);
    double o0_1 = (0.5 * ((x0_0 * ((x1_1 + x1_6) - x1_1)) + (x0_1 * ((x1_3 + x1_7) - x1_7)) + (x0_2 * ((x1_4 + x1_8) - x1_13))));
    st(0, 1, o0_1);
    double o0_7 = (0.5 * ((x0_1 * ((x1_1 + x1_6) - x1_1)) + (x0_3 * ((x1_3 + x1_7) - x1_7)) + (x0_4 * ((x1_4 + x1_8) - x1_13))));
    st(0, 7, o0_7);
    double o0_13 = (0.5 * ((x0_2 * ((x1_1 + x1_6) - x1_1)) + (x0_4 * ((x1_3 + x1_7) - x1_7)) + (x0_5 * ((x1_4 + x1_8) - x1_13))));
    st(0, 13, o0_13);
    double o0_3 = (0.5 * ((x0_0 * ((x1_7 + x1_7) - x1_3)) + (x0_1 * ((x1_9 + x1_9) - x1_9)) + (x0_2 * ((x1_10 + x1_10) - x1_15))));
    st(0, 3, o0_3);
    double o0_9 = (0.5 * ((x0_1 * ((x1_7 + x1_7) - x1_3)) + (x0_3 * ((x1_9 + x1_9) - x1_9)) + (x0_4 * ((x1_10 + x1_10) - x1_15))));
    st(0, 9, o0_9);
    double o0_15 = (0.5 * ((x0_2 * ((x1_7 + x1_7) - x1_3)) + (x0_4 * ((x1_9 + x1_9) - x1_9)) + (x0_5 * ((x1_10 + x1_10) - x1_15))));
    st(0, 15, o0_15);
    double o0_2 = (0.5 * ((x0_0 * ((x1_2 + x1_12) - x1_2)) + (x0_1 * ((x1_4 + x1_13) - x1_8)) + (x0_2 * ((x1_5 + x1_14) - x1_14))));
    st(0, 2, o0_2);
    double o0_8 = (0.5 * ((x0_1 * ((x1_2 + x1_12) - x1_2)) + (x0_3 * ((x1_4 + x1_13) - x1_8)) + (x0_4 * ((x1_5 + x1_14) - x1_14))));
    st(0, 8, o0_8);
    double o0_14 = (0.5 * ((x0_2 * ((x1_2 + x1_12) - x1_2)) + (x0_4 * ((x1_4 + x1_13) - x1_8)) + (x0_5 * ((x1_5 + x1_14) - x1_14))));
    st(0, 14, o0_14);
    double o0_4 = (0.5 * ((x0_0 * ((x1_8 + x1_13) - x1_4)) + (x0_1 * ((x1_10 + x1_15) - x1_10)) + (x0_2 * ((x1_11 + x1_16) - x1_16))));
    st(0, 4, o0_4);
    double o0_10 = (0.5 * ((x0_1 * ((x1_8 + x1_13) - x1_4)) + (x0_3 * ((x1_10 + x1_15) - x1_10)) + (x0_4 * ((x1_11 + x1_16) - x1_16))));
    st(0, 10, o0_10);
    double o0_16 = (0.5 * ((x0_2 * ((x1_8 + x1_13) - x1_4)) + (x0_4 * ((x1_10 + x1_15) - x1_10)) + (x0_5 * ((x1_11 + x1_16) - x1_16))));
    st(0, 16, o0_16);
    double o0_5 = (0.5 * ((x0_0 * ((x1_14 + x1_14) - x1_5)) + (x0_1 * ((x1_16 + x1_16) - x1_11)) + (x0_2 * ((x1_17 + x1_17) - x1_17))));
    st(0, 5, o0_5);
    double o0_11 = (0.5 * ((x0_1 * ((x1_14 + x1_14) - x1_5)) + (x0_3 * ((x1_16 + x1_16) - x1_11)) + (x0_4 * ((x1_17 + x1_17) - x1_17))));
    st(0, 11, o0_11);
    double o0_17 = (0.5 * ((x0_2 * ((x1_14 + x1_14) - x1_5)) + (x0_4 * ((x1_16 + x1_16) - x1_11)) + (x0_5 * ((x1_17 + x1_17) - x1_17))));
    st(0, 17, o0_17);
  }
};

// cov_deriv: covariant derivative of the shift (Sec. 1, footnote)
struct Gen_cov_deriv {
  static constexpr bool kStream = true;
  static constexpr int NF_IN = 3, NF_OUT = 1;
  static constexpr int fin[NF_IN] = {9, 18, 3};
  static constexpr int fout[NF_OUT] = {9};
  static constexpr int NIN = 30, NOUT = 9;
  template <class L, class S>
  __device__ static inline void stream(L&& ld, S&& st) {
    const double x0_0 = ld(0, 0);
    const double x0_1 = ld(0, 1);
    const double x0_2 = ld(0, 2);
    const double x0_3 = ld(0, 3);
    const double x0_4 = ld(0, 4);
    const double x0_5 = ld(0, 5);
    const double x0_6 = ld(0, 6);
    const double x0_7 = ld(0, 7);
    const double x0_8 = ld(0, 8);
    const double x1_0 = ld(1, 0);
    const double x1_1 = ld(1, 1);
    const double x1_2 = ld(1, 2);
    const double x1_3 = ld(1, 3);
    const double x1_4 = ld(1, 4);
    const double x1_5 = ld(1, 5);
    const double x1_6 = ld(1, 6);
    const double x1_7 = ld(1, 7);
    const double x1_8 = ld(1, 8);
    const double x1_9 = ld(1, 9);
    const double x1_10 = ld(1, 10);
    const double x1_11 = ld(1, 11);
    const double x1_12 = ld(1, 12);
    const double x1_13 = ld(1, 13);
    const double x1_14 = ld(1, 14);
    const double x1_15 = ld(1, 15);
    const double x1_16 = ld(1, 16);
    const double x1_17 = ld(1, 17);
    const double x2_0 = ld(2, 0);
    const double x2_1 = ld(2, 1);
    const double x2_2 = ld(2, 2);
    // nabla(j,i) = (dbeta(j,i) - Sum(k, (Gamma(k,i,j) * beta(k))))
    double o0_0 = (x0_0 - ((x1_0 * x2_0) + (x1_6 * x2_1) + (x1_12 * x2_2)));
    st(0, 0, o0_0);
    double o0_1 = (x0_1 - ((x1_1 * x2_0) + (x1_7 * x2_1) + (x1_13 * x2_2)));
    st(0, 1, o0_1);
    double o0_2 = (x0_2 - ((x1_2 * x2_0) + (x1_8 * x2_1) + (x1_14 * x2_2)));
    st(0, 2, o0_2);
    double o0_3 = (x0_3 - ((x1_1 * x2_0) + (x1_7 * x2_1) + (x1_13 * x2_2)));
    st(0, 3, o0_3);
    double o0_4 = (x0_4 - ((x1_3 * x2_0) + (x1_9 * x2_1) + (x1_15 * x2_2)));
    st(0, 4, o0_4);
    double o0_5 = (x0_5 - ((x1_4 * x2_0) + (x1_10 * x2_1) + (x1_16 * x2_2)));
    st(0, 5, o0_5);
    double o0_6 = (x0_6 - ((x1_2 * x2_0) + (x1_8 * x2_1) + (x1_14 * x2_2)));
    st(0, 6, o0_6);
    double o0_7 = (x0_7 - ((x1_4 * x2_0) + (x1_10 * x2_1) + (x1_16 * x2_2)));
    st(0, 7, o0_7);
    double o0_8 = (x0_8 - ((x1_5 * x2_0) + (x1_11 * x2_1) + (x1_17 * x2_2)));
    st(0, 8, o0_8);
  }
};

// dtg: metric evolution from nabla beta (Sec. 1, eq:dtg_ij)
struct Gen_dtg {
  static constexpr bool kStream = true;
  static constexpr int NF_IN = 3, NF_OUT = 1;
  static constexpr int fin[NF_IN] = {1, 6, 9};
  static constexpr int fout[NF_OUT] = {6};
  static constexpr int NIN = 16, NOUT = 6;
  template <class L, class S>
  __device__ static inline void stream(L&& ld, S&& st) {
    const double x0_0 = ld(0, 0);
    const double x1_0 = ld(1, 0);
    const double x1_1 = ld(1, 1);
    const double x1_2 = ld(1, 2);
    const double x1_3 = ld(1, 3);
    const double x1_4 = ld(1, 4);
    const double x1_5 = ld(1, 5);
    const double x2_0 = ld(2, 0);
    const double x2_1 = ld(2, 1);
    const double x2_2 = ld(2, 2);
    const double x2_3 = ld(2, 3);
    const double x2_4 = ld(2, 4);
    const double x2_5 = ld(2, 5);
    const double x2_6 = ld(2, 6);
    const double x2_7 = ld(2, 7);
    const double x2_8 = ld(2, 8);
    // dtg(i,j) = ((((-2.0 * alpha()) * K(i,j)) + nabla(i,j)) + nabla(j,i))
    double o0_0 = ((((-2.0 * x0_0) * x1_0) + x2_0) + x2_0);
    st(0, 0, o0_0);
    double o0_1 = ((((-2.0 * x0_0) * x1_1) + x2_3) + x2_1);
    st(0, 1, o0_1);
    double o0_3 = ((((-2.0 * x0_0) * x1_3) + x2_4) + x2_4);
    st(0, 3, o0_3);
    double o0_2 = ((((-2.0 * x0_0) * x1_2) + x2_6) + x2_2);
    st(0, 2, o0_2);
    double o0_4 = ((((-2.0 * x0_0) * x1_4) + x2_7) + x2_5);
    st(0, 4, o0_4);
    double o0_5 = ((((-2.0 * x0_0) * x1_5) + x2_8) + x2_8);
    st(0, 5, o0_5);
  }
};

// dtg_chain_invg: Christoffel symbols, covariant derivative and metric evolution in one kernel, Gamma and nabla beta in registers (Sec. 1)
struct Gen_dtg_chain_invg {
  static constexpr bool kStream = true;
  static constexpr int NF_IN = 6, NF_OUT = 1;
  static constexpr int fin[NF_IN] = {6, 18, 9, 3, 1, 6};
  static constexpr int fout[NF_OUT] = {6};
  static constexpr int NIN = 43, NOUT = 6;
  template <class L, class S>
  __device__ static inline void stream(L&& ld, S&& st) {
    double t_Gamma[18];
    double t_nabla[9];
    const double x0_0 = ld(0, 0);
    const double x0_1 = ld(0, 1);
    const double x0_2 = ld(0, 2);
    const double x0_3 = ld(0, 3);
    const double x0_4 = ld(0, 4);
    const double x0_5 = ld(0, 5);
    const double x1_0 = ld(1, 0);
    const double x1_1 = ld(1, 1);
    const double x1_2 = ld(1, 2);
    const double x1_3 = ld(1, 3);
    const double x1_4 = ld(1, 4);
    const double x1_5 = ld(1, 5);
    const double x1_6 = ld(1, 6);
    const double x1_7 = ld(1, 7);
    const double x1_8 = ld(1, 8);
    const double x1_9 = ld(1, 9);
    const double x1_10 = ld(1, 10);
    const double x1_11 = ld(1, 11);
    const double x1_12 = ld(1, 12);
    const double x1_13 = ld(1, 13);
    const double x1_14 = ld(1, 14);
    const double x1_15 = ld(1, 15);
    const double x1_16 = ld(1, 16);
    const double x1_17 = ld(1, 17);
    const double x2_0 = ld(2, 0);
    const double x2_1 = ld(2, 1);
    const double x2_2 = ld(2, 2);
    const double x2_3 = ld(2, 3);
    const double x2_4 = ld(2, 4);
    const double x2_5 = ld(2, 5);
    const double x2_6 = ld(2, 6);
    const double x2_7 = ld(2, 7);
    const double x2_8 = ld(2, 8);
    const double x3_0 = ld(3, 0);
    const double x3_1 = ld(3, 1);
    const double x3_2 = ld(3, 2);
    const double x4_0 = ld(4, 0);
    const double x5_0 = ld(5, 0);
    const double x5_1 = ld(5, 1);
    const double x5_2 = ld(5, 2);
    const double x5_3 = ld(5, 3);
    const double x5_4 = ld(5, 4);
    const double x5_5 = ld(5, 5);
    // Gamma(i,j,k) = (0.5 * Sum(l, (Invg(i,l) * ((dg(k,j,l) + dg(j,l,k)) - dg(l,j,k)))))
    t_Gamma[0] = (0.5 * ((x0_0 * ((x1_0 + x1_0) - x1_0)) + (x0_1 * ((x1_1 + x1_1) - x1_6)) + (x0_2 * ((x1_2 + x1_2) - x1_12))));
    t_Gamma[6] = (0.5 * ((x0_1 * ((x1_0 + x1_0) - x1_0)) + (x0_3 * ((x1_1 + x1_1) - x1_6)) + (x0_4 * ((x1_2 + x1_2) - x1_12))));
    t_Gamma[12] = (0.5 * ((x0_2 * ((x1_0 + x1_0) - x1_0)) + (x0_4 * ((x1_1 + x1_1) - x1_6)) + (x0_5 * ((x1_2 + x1_2) - x1_12))));
    t_Gamma[1] = (0.5 * ((x0_0 * ((x1_1 + x1_6) - x1_1)) + (x0_1 * ((x1_3 + x1_7) - x1_7)) + (x0_2 * ((x1_4 + x1_8) - x1_13))));
    t_Gamma[7] = (0.5 * ((x0_1 * ((x1_1 + x1_6) - x1_1)) + (x0_3 * ((x1_3 + x1_7) - x1_7)) + (x0_4 * ((x1_4 + x1_8) - x1_13))));
    t_Gamma[13] = (0.5 * ((x0_2 * ((x1_1 + x1_6) - x1_1)) + (x0_4 * ((x1_3 + x1_7) - x1_7)) + (x0_5 * ((x1_4 + x1_8) - x1_13))));
    t_Gamma[3] = (0.5 * ((x0_0 * ((x1_7 + x1_7) - x1_3)) + (x0_1 * ((x1_9 + x1_9) - x1_9)) + (x0_2 * ((x1_10 + x1_10) - x1_15))));
    t_Gamma[9] = (0.5 * ((x0_1 * ((x1_7 + x1_7) - x1_3)) + (x0_3 * ((x1_9 + x1_9) - x1_9)) + (x0_4 * ((x1_10 + x1_10) - x1_15))));
    t_Gamma[15] = (0.5 * ((x0_2 * ((x1_7 + x1_7) - x1_3)) + (x0_4 * ((x1_9 + x1_9) - x1_9)) + (x0_5 * ((x1_10 + x1_10) - x1_15))));
    t_Gamma[2] = (0.5 * ((x0_0 * ((x1_2 + x1_12) - x1_2)) + (x0_1 * ((x1_4 + x1_13) - x1_8)) + (x0_2 * ((x1_5 + x1_14) - x1_14))));
    t_Gamma[8] = (0.5 * ((x0_1 * ((x1_2 + x1_12) - x1_2)) + (x0_3 * ((x1_4 + x1_13) - x1_8)) + (x0_4 * ((x1_5 + x1_14) - x1_14))));
    t_Gamma[14] = (0.5 * ((x0_2 * ((x1_2 + x1_12) - x1_2)) + (x0_4 * ((x1_4 + x1_13) - x1_8)) + (x0_5 * ((x1_5 + x1_14) - x1_14))));
    t_Gamma[4] = (0.5 * ((x0_0 * ((x1_8 + x1_13) - x1_4)) + (x0_1 * ((x1_10 + x1_15) - x1_10)) + (x0_2 * ((x1_11 + x1_16) - x1_16))));
    t_Gamma[10] = (0.5 * ((x0_1 * ((x1_8 + x1_13) - x1_4)) + (x0_3 * ((x1_10 + x1_15) - x1_10)) + (x0_4 * ((x1_11 + x1_16) - x1_16))));
    t_Gamma[16] = (0.5 * ((x0_2 * ((x1_8 + x1_13) - x1_4)) + (x0_4 * ((x1_10 + x1_15) - x1_10)) + (x0_5 * ((x1_11 + x1_16) - x1_16))));
    t_Gamma[5] = (0.5 * ((x0_0 * ((x1_14 + x1_14) - x1_5)) + (x0_1 * ((x1_16 + x1_16) - x1_11)) + (x0_2 * ((x1_17 + x1_17) - x1_17))));
    t_Gamma[11] = (0.5 * ((x0_1 * ((x1_14 + x1_14) - x1_5)) + (x0_3 * ((x1_16 + x1_16) - x1_11)) + (x0_4 * ((x1_17 + x1_17) - x1_17))));
    t_Gamma[17] = (0.5 * ((x0_2 * ((x1_14 + x1_14) - x1_5)) + (x0_4 * ((x1_16 + x1_16) - x1_11)) + (x0_5 * ((x1_17 + x1_17) - x1_17))));
    // nabla(j,i) = (dbeta(j,i) - Sum(k, (Gamma(k,i,j) * beta(k))))
    t_nabla[0] = (x2_0 - ((t_Gamma[0] * x3_0) + (t_Gamma[6] * x3_1) + (t_Gamma[12] * x3_2)));
    t_nabla[1] = (x2_1 - ((t_Gamma[1] * x3_0) + (t_Gamma[7] * x3_1) + (t_Gamma[13] * x3_2)));
    t_nabla[2] = (x2_2 - ((t_Gamma[2] * x3_0) + (t_Gamma[8] * x3_1) + (t_Gamma[14] * x3_2)));
    t_nabla[3] = (x2_3 - ((t_Gamma[1] * x3_0) + (t_Gamma[7] * x3_1) + (t_Gamma[13] * x3_2)));
    t_nabla[4] = (x2_4 - ((t_Gamma[3] * x3_0) + (t_Gamma[9] * x3_1) + (t_Gamma[15] * x3_2)));
    t_nabla[5] = (x2_5 - ((t_Gamma[4] * x3_0) + (t_Gamma[10] * x3_1) + (t_Gamma[16] * x3_2)));
    t_nabla[6] = (x2_6 - ((t_Gamma[2] * x3_0) + (t_Gamma[8] * x3_1) + (t_Gamma[14] * x3_2)));
    t_nabla[7] = (x2_7 - ((t_Gamma[4] * x3_0) + (t_Gamma[10] * x3_1) + (t_Gamma[16] * x3_2)));
    t_nabla[8] = (x2_8 - ((t_Gamma[5] * x3_0) + (t_Gamma[11] * x3_1) + (t_Gamma[17] * x3_2)));
    // dtg(i,j) = ((((-2.0 * alpha()) * K(i,j)) + nabla(i,j)) + nabla(j,i))
    double o0_0 = ((((-2.0 * x4_0) * x5_0) + t_nabla[0]) + t_nabla[0]);
    st(0, 0, o0_0);
    double o0_1 = ((((-2.0 * x4_0) * x5_1) + t_nabla[3]) + t_nabla[1]);
    st(0, 1, o0_1);
    double o0_3 = ((((-2.0 * x4_0) * x5_3) + t_nabla[4]) + t_nabla[4]);
    st(0, 3, o0_3);
    double o0_2 = ((((-2.0 * x4_0) * x5_2) + t_nabla[6]) + t_nabla[2]);
    st(0, 2, o0_2);
    double o0_4 = ((((-2.0 * x4_0) * x5_4) + t_nabla[7]) + t_nabla[5]);
    st(0, 4, o0_4);
    double o0_5 = ((((-2.0 * x4_0) * x5_5) + t_nabla[8]) + t_nabla[8]);
    st(0, 5, o0_5);
  }
};

// kij: K_ij = 2 alpha g_ij + beta_i beta_j (Sec. 5.1, eq:Kij)
struct Gen_kij {
  static constexpr bool kStream = true;
  static constexpr int NF_IN = 3, NF_OUT = 1;
  static constexpr int fin[NF_IN] = {1, 6, 3};
  static constexpr int fout[NF_OUT] = {6};
  static constexpr int NIN = 10, NOUT = 6;
  template <class L, class S>
  __device__ static inline void stream(L&& ld, S&& st) {
    const double x0_0 = ld(0, 0);
    const double x1_0 = ld(1, 0);
    const double x1_1 = ld(1, 1);
    const double x1_2 = ld(1, 2);
    const double x1_3 = ld(1, 3);
    const double x1_4 = ld(1, 4);
    const double x1_5 = ld(1, 5);
    const double x2_0 = ld(2, 0);
    const double x2_1 = ld(2, 1);
    const double x2_2 = ld(2, 2);
    // K(i,j) = (((2.0 * alpha()) * g(i,j)) + (beta(i) * beta(j)))
    double o0_0 = (((2.0 * x0_0) * x1_0) + (x2_0 * x2_0));
    st(0, 0, o0_0);
    double o0_1 = (((2.0 * x0_0) * x1_1) + (x2_1 * x2_0));
    st(0, 1, o0_1);
    double o0_3 = (((2.0 * x0_0) * x1_3) + (x2_1 * x2_1));
    st(0, 3, o0_3);
    double o0_2 = (((2.0 * x0_0) * x1_2) + (x2_2 * x2_0));
    st(0, 2, o0_2);
    double o0_4 = (((2.0 * x0_0) * x1_4) + (x2_2 * x2_1));
    st(0, 4, o0_4);
    double o0_5 = (((2.0 * x0_0) * x1_5) + (x2_2 * x2_2));
    st(0, 5, o0_5);
  }
};

// assign1: A_i = B_i (Sec. 5.1, eq:Assign1)
struct Gen_assign1 {
  static constexpr bool kStream = true;
  static constexpr int NF_IN = 1, NF_OUT = 1;
  static constexpr int fin[NF_IN] = {3};
  static constexpr int fout[NF_OUT] = {3};
  static constexpr int NIN = 3, NOUT = 3;
  template <class L, class S>
  __device__ static inline void stream(L&& ld, S&& st) {
    const double x0_0 = ld(0, 0);
    const double x0_1 = ld(0, 1);
    const double x0_2 = ld(0, 2);
    // A(i) = B(i)
    double o0_0 = x0_0;
    st(0, 0, o0_0);
    double o0_1 = x0_1;
    st(0, 1, o0_1);
    double o0_2 = x0_2;
    st(0, 2, o0_2);
  }
};

// assign2: A_ij = B_ij (Sec. 5.1, eq:Assign2)
struct Gen_assign2 {
  static constexpr bool kStream = true;
  static constexpr int NF_IN = 1, NF_OUT = 1;
  static constexpr int fin[NF_IN] = {9};
  static constexpr int fout[NF_OUT] = {9};
  static constexpr int NIN = 9, NOUT = 9;
  template <class L, class S>
  __device__ static inline void stream(L&& ld, S&& st) {
    const double x0_0 = ld(0, 0);
    const double x0_1 = ld(0, 1);
    const double x0_2 = ld(0, 2);
    const double x0_3 = ld(0, 3);
    const double x0_4 = ld(0, 4);
    const double x0_5 = ld(0, 5);
    const double x0_6 = ld(0, 6);
    const double x0_7 = ld(0, 7);
    const double x0_8 = ld(0, 8);
    // A(i,j) = B(i,j)
    double o0_0 = x0_0;
    st(0, 0, o0_0);
    double o0_1 = x0_1;
    st(0, 1, o0_1);
    double o0_2 = x0_2;
    st(0, 2, o0_2);
    double o0_3 = x0_3;
    st(0, 3, o0_3);
    double o0_4 = x0_4;
    st(0, 4, o0_4);
    double o0_5 = x0_5;
    st(0, 5, o0_5);
    double o0_6 = x0_6;
    st(0, 6, o0_6);
    double o0_7 = x0_7;
    st(0, 7, o0_7);
    double o0_8 = x0_8;
    st(0, 8, o0_8);
  }
};

// assign3: A_ijk = B_ijk (Sec. 5.1, eq:Assign3)
struct Gen_assign3 {
  static constexpr bool kStream = true;
  static constexpr int NF_IN = 1, NF_OUT = 1;
  static constexpr int fin[NF_IN] = {27};
  static constexpr int fout[NF_OUT] = {27};
  static constexpr int NIN = 27, NOUT = 27;
  template <class L, class S>
  __device__ static inline void stream(L&& ld, S&& st) {
    const double x0_0 = ld(0, 0);
    const double x0_1 = ld(0, 1);
    const double x0_2 = ld(0, 2);
    const double x0_3 = ld(0, 3);
    const double x0_4 = ld(0, 4);
    const double x0_5 = ld(0, 5);
    const double x0_6 = ld(0, 6);
    const double x0_7 = ld(0, 7);
    const double x0_8 = ld(0, 8);
    const double x0_9 = ld(0, 9);
    const double x0_10 = ld(0, 10);
    const double x0_11 = ld(0, 11);
    const double x0_12 = ld(0, 12);
    const double x0_13 = ld(0, 13);
    const double x0_14 = ld(0, 14);
    const double x0_15 = ld(0, 15);
    const double x0_16 = ld(0, 16);
    const double x0_17 = ld(0, 17);
    const double x0_18 = ld(0, 18);
    const double x0_19 = ld(0, 19);
    const double x0_20 = ld(0, 20);
    const double x0_21 = ld(0, 21);
    const double x0_22 = ld(0, 22);
    const double x0_23 = ld(0, 23);
    const double x0_24 = ld(0, 24);
    const double x0_25 = ld(0, 25);
    const double x0_26 = ld(0, 26);
    // A(i,j,k) = B(i,j,k)
    double o0_0 = x0_0;
    st(0, 0, o0_0);
    double o0_1 = x0_1;
    st(0, 1, o0_1);
    double o0_2 = x0_2;
    st(0, 2, o0_2);
    double o0_3 = x0_3;
    st(0, 3, o0_3);
    double o0_4 = x0_4;
    st(0, 4, o0_4);
    double o0_5 = x0_5;
    st(0, 5, o0_5);
    double o0_6 = x0_6;
    st(0, 6, o0_6);
    double o0_7 = x0_7;
    st(0, 7, o0_7);
    double o0_8 = x0_8;
    st(0, 8, o0_8);
    double o0_9 = x0_9;
    st(0, 9, o0_9);
    double o0_10 = x0_10;
    st(0, 10, o0_10);
    double o0_11 = x0_11;
    st(0, 11, o0_11);
    double o0_12 = x0_12;
    st(0, 12, o0_12);
    double o0_13 = x0_13;
    st(0, 13, o0_13);
    double o0_14 = x0_14;
    st(0, 14, o0_14);
    double o0_15 = x0_15;
    st(0, 15, o0_15);
    double o0_16 = x0_16;
    st(0, 16, o0_16);
    double o0_17 = x0_17;
    st(0, 17, o0_17);
    double o0_18 = x0_18;
    st(0, 18, o0_18);
    double o0_19 = x0_19;
    st(0, 19, o0_19);
    double o0_20 = x0_20;
    st(0, 20, o0_20);
    double o0_21 = x0_21;
    st(0, 21, o0_21);
    double o0_22 = x0_22;
    st(0, 22, o0_22);
    double o0_23 = x0_23;
    st(0, 23, o0_23);
    double o0_24 = x0_24;
    st(0, 24, o0_24);
    double o0_25 = x0_25;
    st(0, 25, o0_25);
    double o0_26 = x0_26;
    st(0, 26, o0_26);
  }
};

// add1: A_i = B_i + C_i (Sec. 5.1, eq:Add1)
struct Gen_add1 {
  static constexpr bool kStream = true;
  static constexpr int NF_IN = 2, NF_OUT = 1;
  static constexpr int fin[NF_IN] = {3, 3};
  static constexpr int fout[NF_OUT] = {3};
  static constexpr int NIN = 6, NOUT = 3;
  template <class L, class S>
  __device__ static inline void stream(L&& ld, S&& st) {
    const double x0_0 = ld(0, 0);
    const double x0_1 = ld(0, 1);
    const double x0_2 = ld(0, 2);
    const double x1_0 = ld(1, 0);
    const double x1_1 = ld(1, 1);
    const double x1_2 = ld(1, 2);
    // A(i) = (B(i) + C(i))
    double o0_0 = (x0_0 + x1_0);
    st(0, 0, o0_0);
    double o0_1 = (x0_1 + x1_1);
    st(0, 1, o0_1);
    double o0_2 = (x0_2 + x1_2);
    st(0, 2, o0_2);
  }
};

// add2: A_i = B_i + C_i + D_i (Sec. 5.1, eq:Add2)
struct Gen_add2 {
  static constexpr bool kStream = true;
  static constexpr int NF_IN = 3, NF_OUT = 1;
  static constexpr int fin[NF_IN] = {3, 3, 3};
  static constexpr int fout[NF_OUT] = {3};
  static constexpr int NIN = 9, NOUT = 3;
  template <class L, class S>
  __device__ static inline void stream(L&& ld, S&& st) {
    const double x0_0 = ld(0, 0);
    const double x0_1 = ld(0, 1);
    const double x0_2 = ld(0, 2);
    const double x1_0 = ld(1, 0);
    const double x1_1 = ld(1, 1);
    const double x1_2 = ld(1, 2);
    const double x2_0 = ld(2, 0);
    const double x2_1 = ld(2, 1);
    const double x2_2 = ld(2, 2);
    // A(i) = ((B(i) + C(i)) + D(i))
    double o0_0 = ((x0_0 + x1_0) + x2_0);
    st(0, 0, o0_0);
    double o0_1 = ((x0_1 + x1_1) + x2_1);
    st(0, 1, o0_1);
    double o0_2 = ((x0_2 + x1_2) + x2_2);
    st(0, 2, o0_2);
  }
};

// add3: A_i = B_i + C_i + D_i + E_i (Sec. 5.1, eq:Add3)
struct Gen_add3 {
  static constexpr bool kStream = true;
  static constexpr int NF_IN = 4, NF_OUT = 1;
  static constexpr int fin[NF_IN] = {3, 3, 3, 3};
  static constexpr int fout[NF_OUT] = {3};
  static constexpr int NIN = 12, NOUT = 3;
  template <class L, class S>
  __device__ static inline void stream(L&& ld, S&& st) {
    const double x0_0 = ld(0, 0);
    const double x0_1 = ld(0, 1);
    const double x0_2 = ld(0, 2);
    const double x1_0 = ld(1, 0);
    const double x1_1 = ld(1, 1);
    const double x1_2 = ld(1, 2);
    const double x2_0 = ld(2, 0);
    const double x2_1 = ld(2, 1);
    const double x2_2 = ld(2, 2);
    const double x3_0 = ld(3, 0);
    const double x3_1 = ld(3, 1);
    const double x3_2 = ld(3, 2);
    // A(i) = (((B(i) + C(i)) + D(i)) + E(i))
    double o0_0 = (((x0_0 + x1_0) + x2_0) + x3_0);
    st(0, 0, o0_0);
    double o0_1 = (((x0_1 + x1_1) + x2_1) + x3_1);
    st(0, 1, o0_1);
    double o0_2 = (((x0_2 + x1_2) + x2_2) + x3_2);
    st(0, 2, o0_2);
  }
};

// mult1: A_ij = B_i C_j (Sec. 5.1, eq:Mult1)
struct Gen_mult1 {
  static constexpr bool kStream = true;
  static constexpr int NF_IN = 2, NF_OUT = 1;
  static constexpr int fin[NF_IN] = {3, 3};
  static constexpr int fout[NF_OUT] = {9};
  static constexpr int NIN = 6, NOUT = 9;
  template <class L, class S>
  __device__ static inline void stream(L&& ld, S&& st) {
    const double x0_0 = ld(0, 0);
    const double x0_1 = ld(0, 1);
    const double x0_2 = ld(0, 2);
    const double x1_0 = ld(1, 0);
    const double x1_1 = ld(1, 1);
    const double x1_2 = ld(1, 2);
    // A(i,j) = (B(i) * C(j))
    double o0_0 = (x0_0 * x1_0);
    st(0, 0, o0_0);
    double o0_1 = (x0_0 * x1_1);
    st(0, 1, o0_1);
    double o0_2 = (x0_0 * x1_2);
    st(0, 2, o0_2);
    double o0_3 = (x0_1 * x1_0);
    st(0, 3, o0_3);
    double o0_4 = (x0_1 * x1_1);
    st(0, 4, o0_4);
    double o0_5 = (x0_1 * x1_2);
    st(0, 5, o0_5);
    double o0_6 = (x0_2 * x1_0);
    st(0, 6, o0_6);
    double o0_7 = (x0_2 * x1_1);
    st(0, 7, o0_7);
    double o0_8 = (x0_2 * x1_2);
    st(0, 8, o0_8);
  }
};

// mult2: A_ijk = B_i C_j D_k (Sec. 5.1, eq:Mult2)
struct Gen_mult2 {
  static constexpr bool kStream = true;
  static constexpr int NF_IN = 3, NF_OUT = 1;
  static constexpr int fin[NF_IN] = {3, 3, 3};
  static constexpr int fout[NF_OUT] = {27};
  static constexpr int NIN = 9, NOUT = 27;
  template <class L, class S>
  __device__ static inline void stream(L&& ld, S&& st) {
    const double x0_0 = ld(0, 0);
    const double x0_1 = ld(0, 1);
    const double x0_2 = ld(0, 2);
    const double x1_0 = ld(1, 0);
    const double x1_1 = ld(1, 1);
    const double x1_2 = ld(1, 2);
    const double x2_0 = ld(2, 0);
    const double x2_1 = ld(2, 1);
    const double x2_2 = ld(2, 2);
    // A(i,j,k) = ((B(i) * C(j)) * D(k))
    double o0_0 = ((x0_0 * x1_0) * x2_0);
    st(0, 0, o0_0);
    double o0_1 = ((x0_0 * x1_0) * x2_1);
    st(0, 1, o0_1);
    double o0_2 = ((x0_0 * x1_0) * x2_2);
    st(0, 2, o0_2);
    double o0_3 = ((x0_0 * x1_1) * x2_0);
    st(0, 3, o0_3);
    double o0_4 = ((x0_0 * x1_1) * x2_1);
    st(0, 4, o0_4);
    double o0_5 = ((x0_0 * x1_1) * x2_2);
    st(0, 5, o0_5);
    double o0_6 = ((x0_0 * x1_2) * x2_0);
    st(0, 6, o0_6);
    double o0_7 = ((x0_0 * x1_2) * x2_1);
    st(0, 7, o0_7);
    double o0_8 = ((x0_0 * x1_2) * x2_2);
    st(0, 8, o0_8);
    double o0_9 = ((x0_1 * x1_0) * x2_0);
    st(0, 9, o0_9);
    double o0_10 = ((x0_1 * x1_0) * x2_1);
    st(0, 10, o0_10);
    double o0_11 = ((x0_1 * x1_0) * x2_2);
    st(0, 11, o0_11);
    double o0_12 = ((x0_1 * x1_1) * x2_0);
    st(0, 12, o0_12);
    double o0_13 = ((x0_1 * x1_1) * x2_1);
    st(0, 13, o0_13);
    double o0_14 = ((x0_1 * x1_1) * x2_2);
    st(0, 14, o0_14);
    double o0_15 = ((x0_1 * x1_2) * x2_0);
    st(0, 15, o0_15);
    double o0_16 = ((x0_1 * x1_2) * x2_1);
    st(0, 16, o0_16);
    double o0_17 = ((x0_1 * x1_2) * x2_2);
    st(0, 17, o0_17);
    double o0_18 = ((x0_2 * x1_0) * x2_0);
    st(0, 18, o0_18);
    double o0_19 = ((x0_2 * x1_0) * x2_1);
    st(0, 19, o0_19);
    double o0_20 = ((x0_2 * x1_0) * x2_2);
    st(0, 20, o0_20);
    double o0_21 = ((x0_2 * x1_1) * x2_0);
    st(0, 21, o0_21);
    double o0_22 = ((x0_2 * x1_1) * x2_1);
    st(0, 22, o0_22);
    double o0_23 = ((x0_2 * x1_1) * x2_2);
    st(0, 23, o0_23);
    double o0_24 = ((x0_2 * x1_2) * x2_0);
    st(0, 24, o0_24);
    double o0_25 = ((x0_2 * x1_2) * x2_1);
    st(0, 25, o0_25);
    double o0_26 = ((x0_2 * x1_2) * x2_2);
    st(0, 26, o0_26);
  }
};

// mult3: A_ijkl = B_i C_j D_k E_l (Sec. 5.1, eq:Mult3)
struct Gen_mult3 {
  static constexpr bool kStream = true;
  static constexpr int NF_IN = 4, NF_OUT = 1;
  static constexpr int fin[NF_IN] = {3, 3, 3, 3};
  static constexpr int fout[NF_OUT] = {81};
  static constexpr int NIN = 12, NOUT = 81;
  template <class L, class S>
  __device__ static inline void stream(L&& ld, S&& st) {
    const double x0_0 = ld(0, 0);
    const double x0_1 = ld(0, 1);
    const double x0_2 = ld(0, 2);
    const double x1_0 = ld(1, 0);
    const double x1_1 = ld(1, 1);
    const double x1_2 = ld(1, 2);
    const double x2_0 = ld(2, 0);
    const double x2_1 = ld(2, 1);
    const double x2_2 = ld(2, 2);
    const double x3_0 = ld(3, 0);
    const double x3_1 = ld(3, 1);
    const double x3_2 = ld(3, 2);
    // A(i,j,k,l) = (((B(i) * C(j)) * D(k)) * E(l))
    double o0_0 = (((x0_0 * x1_0) * x2_0) * x3_0);
    st(0, 0, o0_0);
    double o0_1 = (((x0_0 * x1_0) * x2_0) * x3_1);
    st(0, 1, o0_1);
    double o0_2 = (((x0_0 * x1_0) * x2_0) * x3_2);
    st(0, 2, o0_2);
    double o0_3 = (((x0_0 * x1_0) * x2_1) * x3_0);
    st(0, 3, o0_3);
    double o0_4 = (((x0_0 * x1_0) * x2_1) * x3_1);
    st(0, 4, o0_4);
    double o0_5 = (((x0_0 * x1_0) * x2_1) * x3_2);
    st(0, 5, o0_5);
    double o0_6 = (((x0_0 * x1_0) * x2_2) * x3_0);
    st(0, 6, o0_6);
    double o0_7 = (((x0_0 * x1_0) * x2_2) * x3_1);
    st(0, 7, o0_7);
    double o0_8 = (((x0_0 * x1_0) * x2_2) * x3_2);
    st(0, 8, o0_8);
    double o0_9 = (((x0_0 * x1_1) * x2_0) * x3_0);
    st(0, 9, o0_9);
    double o0_10 = (((x0_0 * x1_1) * x2_0) * x3_1);
    st(0, 10, o0_10);
    double o0_11 = (((x0_0 * x1_1) * x2_0) * x3_2);
    st(0, 11, o0_11);
    double o0_12 = (((x0_0 * x1_1) * x2_1) * x3_0);
    st(0, 12, o0_12);
    double o0_13 = (((x0_0 * x1_1) * x2_1) * x3_1);
    st(0, 13, o0_13);
    double o0_14 = (((x0_0 * x1_1) * x2_1) * x3_2);
    st(0, 14, o0_14);
    double o0_15 = (((x0_0 * x1_1) * x2_2) * x3_0);
    st(0, 15, o0_15);
    double o0_16 = (((x0_0 * x1_1) * x2_2) * x3_1);
    st(0, 16, o0_16);
    double o0_17 = (((x0_0 * x1_1) * x2_2) * x3_2);
    st(0, 17, o0_17);
    double o0_18 = (((x0_0 * x1_2) * x2_0) * x3_0);
    st(0, 18, o0_18);
    double o0_19 = (((x0_0 * x1_2) * x2_0) * x3_1);
    st(0, 19, o0_19);
    double o0_20 = (((x0_0 * x1_2) * x2_0) * x3_2);
    st(0, 20, o0_20);
    double o0_21 = (((x0_0 * x1_2) * x2_1) * x3_0);
    st(0, 21, o0_21);
    double o0_22 = (((x0_0 * x1_2) * x2_1) * x3_1);
    st(0, 22, o0_22);
    double o0_23 = (((x0_0 * x1_2) * x2_1) * x3_2);
    st(0, 23, o0_23);
    double o0_24 = (((x0_0 * x1_2) * x2_2) * x3_0);
    st(0, 24, o0_24);
    double o0_25 = (((x0_0 * x1_2) * x2_2) * x3_1);
    st(0, 25, o0_25);
    double o0_26 = (((x0_0 * x1_2) * x2_2) * x3_2);
    st(0, 26, o0_26);
    double o0_27 = (((x0_1 * x1_0) * x2_0) * x3_0);
    st(0, 27, o0_27);
    double o0_28 = (((x0_1 * x1_0) * x2_0) * x3_1);
    st(0, 28, o0_28);
    double o0_29 = (((x0_1 * x1_0) * x2_0) * x3_2);
    st(0, 29, o0_29);
    double o0_30 = (((x0_1 * x1_0) * x2_1) * x3_0);
    st(0, 30, o0_30);
    double o0_31 = (((x0_1 * x1_0) * x2_1) * x3_1);
    st(0, 31, o0_31);
    double o0_32 = (((x0_1 * x1_0) * x2_1) * x3_2);
    st(0, 32, o0_32);
    double o0_33 = (((x0_1 * x1_0) * x2_2) * x3_0);
    st(0, 33, o0_33);
    double o0_34 = (((x0_1 * x1_0) * x2_2) * x3_1);
    st(0, 34, o0_34);
    double o0_35 = (((x0_1 * x1_0) * x2_2) * x3_2);
    st(0, 35, o0_35);
    double o0_36 = (((x0_1 * x1_1) * x2_0) * x3_0);
    st(0, 36, o0_36);
    double o0_37 = (((x0_1 * x1_1) * x2_0) * x3_1);
    st(0, 37, o0_37);
    double o0_38 = (((x0_1 * x1_1) * x2_0) * x3_2);
    st(0, 38, o0_38);
    double o0_39 = (((x0_1 * x1_1) * x2_1) * x3_0);
    st(0, 39, o0_39);
    double o0_40 = (((x0_1 * x1_1) * x2_1) * x3_1);
    st(0, 40, o0_40);
    double o0_41 = (((x0_1 * x1_1) * x2_1) * x3_2);
    st(0, 41, o0_41);
    double o0_42 = (((x0_1 * x1_1) * x2_2) * x3_0);
    st(0, 42, o0_42);
    double o0_43 = (((x0_1 * x1_1) * x2_2) * x3_1);
    st(0, 43, o0_43);
    double o0_44 = (((x0_1 * x1_1) * x2_2) * x3_2);
    st(0, 44, o0_44);
    double o0_45 = (((x0_1 * x1_2) * x2_0) * x3_0);
    st(0, 45, o0_45);
    double o0_46 = (((x0_1 * x1_2) * x2_0) * x3_1);
    st(0, 46, o0_46);
    double o0_47 = (((x0_1 * x1_2) * x2_0) * x3_2);
    st(0, 47, o0_47);
    double o0_48 = (((x0_1 * x1_2) * x2_1) * x3_0);
    st(0, 48, o0_48);
    double o0_49 = (((x0_1 * x1_2) * x2_1) * x3_1);
    st(0, 49, o0_49);
    double o0_50 = (((x0_1 * x1_2) * x2_1) * x3_2);
    st(0, 50, o0_50);
    double o0_51 = (((x0_1 * x1_2) * x2_2) * x3_0);
    st(0, 51, o0_51);
    double o0_52 = (((x0_1 * x1_2) * x2_2) * x3_1);
    st(0, 52, o0_52);
    double o0_53 = (((x0_1 * x1_2) * x2_2) * x3_2);
    st(0, 53, o0_53);
    double o0_54 = (((x0_2 * x1_0) * x2_0) * x3_0);
    st(0, 54, o0_54);
    double o0_55 = (((x0_2 * x1_0) * x2_0) * x3_1);
    st(0, 55, o0_55);
    double o0_56 = (((x0_2 * x1_0) * x2_0) * x3_2);
    st(0, 56, o0_56);
    double o0_57 = (((x0_2 * x1_0) * x2_1) * x3_0);
    st(0, 57, o0_57);
    double o0_58 = (((x0_2 * x1_0) * x2_1) * x3_1);
    st(0, 58, o0_58);
    double o0_59 = (((x0_2 * x1_0) * x2_1) * x3_2);
    st(0, 59, o0_59);
    double o0_60 = (((x0_2 * x1_0) * x2_2) * x3_0);
    st(0, 60, o0_60);
    double o0_61 = (((x0_2 * x1_0) * x2_2) * x3_1);
    st(0, 61, o0_61);
    double o0_62 = (((x0_2 * x1_0) * x2_2) * x3_2);
    st(0, 62, o0_62);
    double o0_63 = (((x0_2 * x1_1) * x2_0) * x3_0);
    st(0, 63, o0_63);
    double o0_64 = (((x0_2 * x1_1) * x2_0) * x3_1);
    st(0, 64, o0_64);
    double o0_65 = (((x0_2 * x1_1) * x2_0) * x3_2);
    st(0, 65, o0_65);
    double o0_66 = (((x0_2 * x1_1) * x2_1) * x3_0);
    st(0, 66, o0_66);
    double o0_67 = (((x0_2 * x1_1) * x2_1) * x3_1);
    st(0, 67, o0_67);
    double o0_68 = (((x0_2 * x1_1) * x2_1) * x3_2);
    st(0, 68, o0_68);
    double o0_69 = (((x0_2 * x1_1) * x2_2) * x3_0);
    st(0, 69, o0_69);
    double o0_70 = (((x0_2 * x1_1) * x2_2) * x3_1);
    st(0, 70, o0_70);
    double o0_71 = (((x0_2 * x1_1) * x2_2) * x3_2);
    st(0, 71, o0_71);
    double o0_72 = (((x0_2 * x1_2) * x2_0) * x3_0);
    st(0, 72, o0_72);
    double o0_73 = (((x0_2 * x1_2) * x2_0) * x3_1);
    st(0, 73, o0_73);
    double o0_74 = (((x0_2 * x1_2) * x2_0) * x3_2);
    st(0, 74, o0_74);
    double o0_75 = (((x0_2 * x1_2) * x2_1) * x3_0);
    st(0, 75, o0_75);
    double o0_76 = (((x0_2 * x1_2) * x2_1) * x3_1);
    st(0, 76, o0_76);
    double o0_77 = (((x0_2 * x1_2) * x2_1) * x3_2);
    st(0, 77, o0_77);
    double o0_78 = (((x0_2 * x1_2) * x2_2) * x3_0);
    st(0, 78, o0_78);
    double o0_79 = (((x0_2 * x1_2) * x2_2) * x3_1);
    st(0, 79, o0_79);
    double o0_80 = (((x0_2 * x1_2) * x2_2) * x3_2);
    st(0, 80, o0_80);
  }
};

// contract1: A_ijkl = B_i^m E_mjkl (Sec. 5.1, eq:Contract1)
struct Gen_contract1 {
  static constexpr bool kStream = true;
  static constexpr int NF_IN = 2, NF_OUT = 1;
  static constexpr int fin[NF_IN] = {9, 81};
  static constexpr int fout[NF_OUT] = {81};
  static constexpr int NIN = 90, NOUT = 81;
  template <class L, class S>
  __device__ static inline void stream(L&& ld, S&& st) {
    // A(i,j,k,l) = Sum(m, (B(i,m) * E(m,j,k,l)))
    const double x0_0 = ld(0, 0);
    const double x1_0 = ld(1, 0);
    const double x0_1 = ld(0, 1);
    const double x1_27 = ld(1, 27);
    const double x0_2 = ld(0, 2);
    const double x1_54 = ld(1, 54);
    double o0_0 = ((x0_0 * x1_0) + (x0_1 * x1_27) + (x0_2 * x1_54));
    st(0, 0, o0_0);
    const double x0_3 = ld(0, 3);
    const double x0_4 = ld(0, 4);
    const double x0_5 = ld(0, 5);
    double o0_27 = ((x0_3 * x1_0) + (x0_4 * x1_27) + (x0_5 * x1_54));
    st(0, 27, o0_27);
    const double x0_6 = ld(0, 6);
    const double x0_7 = ld(0, 7);
    const double x0_8 = ld(0, 8);
    double o0_54 = ((x0_6 * x1_0) + (x0_7 * x1_27) + (x0_8 * x1_54));
    st(0, 54, o0_54);
    const double x1_1 = ld(1, 1);
    const double x1_28 = ld(1, 28);
    const double x1_55 = ld(1, 55);
    double o0_1 = ((x0_0 * x1_1) + (x0_1 * x1_28) + (x0_2 * x1_55));
    st(0, 1, o0_1);
    double o0_28 = ((x0_3 * x1_1) + (x0_4 * x1_28) + (x0_5 * x1_55));
    st(0, 28, o0_28);
    double o0_55 = ((x0_6 * x1_1) + (x0_7 * x1_28) + (x0_8 * x1_55));
    st(0, 55, o0_55);
    const double x1_2 = ld(1, 2);
    const double x1_29 = ld(1, 29);
    const double x1_56 = ld(1, 56);
    double o0_2 = ((x0_0 * x1_2) + (x0_1 * x1_29) + (x0_2 * x1_56));
    st(0, 2, o0_2);
    double o0_29 = ((x0_3 * x1_2) + (x0_4 * x1_29) + (x0_5 * x1_56));
    st(0, 29, o0_29);
    double o0_56 = ((x0_6 * x1_2) + (x0_7 * x1_29) + (x0_8 * x1_56));
    st(0, 56, o0_56);
    const double x1_3 = ld(1, 3);
    const double x1_30 = ld(1, 30);
    const double x1_57 = ld(1, 57);
    double o0_3 = ((x0_0 * x1_3) + (x0_1 * x1_30) + (x0_2 * x1_57));
    st(0, 3, o0_3);
    double o0_30 = ((x0_3 * x1_3) + (x0_4 * x1_30) + (x0_5 * x1_57));
    st(0, 30, o0_30);
    double o0_57 = ((x0_6 * x1_3) + (x0_7 * x1_30) + (x0_8 * x1_57));
    st(0, 57, o0_57);
    const double x1_4 = ld(1, 4);
    const double x1_31 = ld(1, 31);
    const double x1_58 = ld(1, 58);
    double o0_4 = ((x0_0 * x1_4) + (x0_1 * x1_31) + (x0_2 * x1_58));
    st(0, 4, o0_4);
    double o0_31 = ((x0_3 * x1_4) + (x0_4 * x1_31) + (x0_5 * x1_58));
    st(0, 31, o0_31);
    double o0_58 = ((x0_6 * x1_4) + (x0_7 * x1_31) + (x0_8 * x1_58));
    st(0, 58, o0_58);
    const double x1_5 = ld(1, 5);
    const double x1_32 = ld(1, 32);
    const double x1_59 = ld(1, 59);
    double o0_5 = ((x0_0 * x1_5) + (x0_1 * x1_32) + (x0_2 * x1_59));
    st(0, 5, o0_5);
    double o0_32 = ((x0_3 * x1_5) + (x0_4 * x1_32) + (x0_5 * x1_59));
    st(0, 32, o0_32);
    double o0_59 = ((x0_6 * x1_5) + (x0_7 * x1_32) + (x0_8 * x1_59));
    st(0, 59, o0_59);
    const double x1_6 = ld(1, 6);
    const double x1_33 = ld(1, 33);
    const double x1_60 = ld(1, 60);
    double o0_6 = ((x0_0 * x1_6) + (x0_1 * x1_33) + (x0_2 * x1_60));
    st(0, 6, o0_6);
    double o0_33 = ((x0_3 * x1_6) + (x0_4 * x1_33) + (x0_5 * x1_60));
    st(0, 33, o0_33);
    double o0_60 = ((x0_6 * x1_6) + (x0_7 * x1_33) + (x0_8 * x1_60));
    st(0, 60, o0_60);
    const double x1_7 = ld(1, 7);
    const double x1_34 = ld(1, 34);
    const double x1_61 = ld(1, 61);
    double o0_7 = ((x0_0 * x1_7) + (x0_1 * x1_34) + (x0_2 * x1_61));
    st(0, 7, o0_7);
    double o0_34 = ((x0_3 * x1_7) + (x0_4 * x1_34) + (x0_5 * x1_61));
    st(0, 34, o0_34);
    double o0_61 = ((x0_6 * x1_7) + (x0_7 * x1_34) + (x0_8 * x1_61));
    st(0, 61, o0_61);
    const double x1_8 = ld(1, 8);
    const double x1_35 = ld(1, 35);
    const double x1_62 = ld(1, 62);
    double o0_8 = ((x0_0 * x1_8) + (x0_1 * x1_35) + (x0_2 * x1_62));
    st(0, 8, o0_8);
    double o0_35 = ((x0_3 * x1_8) + (x0_4 * x1_35) + (x0_5 * x1_62));
    st(0, 35, o0_35);
    double o0_62 = ((x0_6 * x1_8) + (x0_7 * x1_35) + (x0_8 * x1_62));
    st(0, 62, o0_62);
    __builtin_amdgcn_sched_barrier(0);
    const double x1_9 = ld(1, 9);
    const double x1_36 = ld(1, 36);
    const double x1_63 = ld(1, 63);
    double o0_9 = ((x0_0 * x1_9) + (x0_1 * x1_36) + (x0_2 * x1_63));
    st(0, 9, o0_9);
    double o0_36 = ((x0_3 * x1_9) + (x0_4 * x1_36) + (x0_5 * x1_63));
    st(0, 36, o0_36);
    double o0_63 = ((x0_6 * x1_9) + (x0_7 * x1_36) + (x0_8 * x1_63));
    st(0, 63, o0_63);
    const double x1_10 = ld(1, 10);
    const double x1_37 = ld(1, 37);
    const double x1_64 = ld(1, 64);
    double o0_10 = ((x0_0 * x1_10) + (x0_1 * x1_37) + (x0_2 * x1_64));
    st(0, 10, o0_10);
    double o0_37 = ((x0_3 * x1_10) + (x0_4 * x1_37) + (x0_5 * x1_64));
    st(0, 37, o0_37);
    double o0_64 = ((x0_6 * x1_10) + (x0_7 * x1_37) + (x0_8 * x1_64));
    st(0, 64, o0_64);
    const double x1_11 = ld(1, 11);
    const double x1_38 = ld(1, 38);
    const double x1_65 = ld(1, 65);
    double o0_11 = ((x0_0 * x1_11) + (x0_1 * x1_38) + (x0_2 * x1_65));
    st(0, 11, o0_11);
    double o0_38 = ((x0_3 * x1_11) + (x0_4 * x1_38) + (x0_5 * x1_65));
    st(0, 38, o0_38);
    double o0_65 = ((x0_6 * x1_11) + (x0_7 * x1_38) + (x0_8 * x1_65));
    st(0, 65, o0_65);
    const double x1_12 = ld(1, 12);
    const double x1_39 = ld(1, 39);
    const double x1_66 = ld(1, 66);
    double o0_12 = ((x0_0 * x1_12) + (x0_1 * x1_39) + (x0_2 * x1_66));
    st(0, 12, o0_12);
    double o0_39 = ((x0_3 * x1_12) + (x0_4 * x1_39) + (x0_5 * x1_66));
    st(0, 39, o0_39);
    double o0_66 = ((x0_6 * x1_12) + (x0_7 * x1_39) + (x0_8 * x1_66));
    st(0, 66, o0_66);
    const double x1_13 = ld(1, 13);
    const double x1_40 = ld(1, 40);
    const double x1_67 = ld(1, 67);
    double o0_13 = ((x0_0 * x1_13) + (x0_1 * x1_40) + (x0_2 * x1_67));
    st(0, 13, o0_13);
    double o0_40 = ((x0_3 * x1_13) + (x0_4 * x1_40) + (x0_5 * x1_67));
    st(0, 40, o0_40);
    double o0_67 = ((x0_6 * x1_13) + (x0_7 * x1_40) + (x0_8 * x1_67));
    st(0, 67, o0_67);
    const double x1_14 = ld(1, 14);
    const double x1_41 = ld(1, 41);
    const double x1_68 = ld(1, 68);
    double o0_14 = ((x0_0 * x1_14) + (x0_1 * x1_41) + (x0_2 * x1_68));
    st(0, 14, o0_14);
    double o0_41 = ((x0_3 * x1_14) + (x0_4 * x1_41) + (x0_5 * x1_68));
    st(0, 41, o0_41);
    double o0_68 = ((x0_6 * x1_14) + (x0_7 * x1_41) + (x0_8 * x1_68));
    st(0, 68, o0_68);
    const double x1_15 = ld(1, 15);
    const double x1_42 = ld(1, 42);
    const double x1_69 = ld(1, 69);
    double o0_15 = ((x0_0 * x1_15) + (x0_1 * x1_42) + (x0_2 * x1_69));
    st(0, 15, o0_15);
    double o0_42 = ((x0_3 * x1_15) + (x0_4 * x1_42) + (x0_5 * x1_69));
    st(0, 42, o0_42);
    double o0_69 = ((x0_6 * x1_15) + (x0_7 * x1_42) + (x0_8 * x1_69));
    st(0, 69, o0_69);
    const double x1_16 = ld(1, 16);
    const double x1_43 = ld(1, 43);
    const double x1_70 = ld(1, 70);
    double o0_16 = ((x0_0 * x1_16) + (x0_1 * x1_43) + (x0_2 * x1_70));
    st(0, 16, o0_16);
    double o0_43 = ((x0_3 * x1_16) + (x0_4 * x1_43) + (x0_5 * x1_70));
    st(0, 43, o0_43);
    double o0_70 = ((x0_6 * x1_16) + (x0_7 * x1_43) + (x0_8 * x1_70));
    st(0, 70, o0_70);
    const double x1_17 = ld(1, 17);
    const double x1_44 = ld(1, 44);
    const double x1_71 = ld(1, 71);
    double o0_17 = ((x0_0 * x1_17) + (x0_1 * x1_44) + (x0_2 * x1_71));
    st(0, 17, o0_17);
    double o0_44 = ((x0_3 * x1_17) + (x0_4 * x1_44) + (x0_5 * x1_71));
    st(0, 44, o0_44);
    double o0_71 = ((x0_6 * x1_17) + (x0_7 * x1_44) + (x0_8 * x1_71));
    st(0, 71, o0_71);
    __builtin_amdgcn_sched_barrier(0);
    const double x1_18 = ld(1, 18);
    const double x1_45 = ld(1, 45);
    const double x1_72 = ld(1, 72);
    double o0_18 = ((x0_0 * x1_18) + (x0_1 * x1_45) + (x0_2 * x1_72));
    st(0, 18, o0_18);
    double o0_45 = ((x0_3 * x1_18) + (x0_4 * x1_45) + (x0_5 * x1_72));
    st(0, 45, o0_45);
    double o0_72 = ((x0_6 * x1_18) + (x0_7 * x1_45) + (x0_8 * x1_72));
    st(0, 72, o0_72);
    const double x1_19 = ld(1, 19);
    const double x1_46 = ld(1, 46);
    const double x1_73 = ld(1, 73);
    double o0_19 = ((x0_0 * x1_19) + (x0_1 * x1_46) + (x0_2 * x1_73));
    st(0, 19, o0_19);
    double o0_46 = ((x0_3 * x1_19) + (x0_4 * x1_46) + (x0_5 * x1_73));
    st(0, 46, o0_46);
    double o0_73 = ((x0_6 * x1_19) + (x0_7 * x1_46) + (x0_8 * x1_73));
    st(0, 73, o0_73);
    const double x1_20 = ld(1, 20);
    const double x1_47 = ld(1, 47);
    const double x1_74 = ld(1, 74);
    double o0_20 = ((x0_0 * x1_20) + (x0_1 * x1_47) + (x0_2 * x1_74));
    st(0, 20, o0_20);
    double o0_47 = ((x0_3 * x1_20) + (x0_4 * x1_47) + (x0_5 * x1_74));
    st(0, 47, o0_47);
    double o0_74 = ((x0_6 * x1_20) + (x0_7 * x1_47) + (x0_8 * x1_74));
    st(0, 74, o0_74);
    const double x1_21 = ld(1, 21);
    const double x1_48 = ld(1, 48);
    const double x1_75 = ld(1, 75);
    double o0_21 = ((x0_0 * x1_21) + (x0_1 * x1_48) + (x0_2 * x1_75));
    st(0, 21, o0_21);
    double o0_48 = ((x0_3 * x1_21) + (x0_4 * x1_48) + (x0_5 * x1_75));
    st(0, 48, o0_48);
    double o0_75 = ((x0_6 * x1_21) + (x0_7 * x1_48) + (x0_8 * x1_75));
    st(0, 75, o0_75);
    const double x1_22 = ld(1, 22);
    const double x1_49 = ld(1, 49);
    const double x1_76 = ld(1, 76);
    double o0_22 = ((x0_0 * x1_22) + (x0_1 * x1_49) + (x0_2 * x1_76));
    st(0, 22, o0_22);
    double o0_49 = ((x0_3 * x1_22) + (x0_4 * x1_49) + (x0_5 * x1_76));
    st(0, 49, o0_49);
    double o0_76 = ((x0_6 * x1_22) + (x0_7 * x1_49) + (x0_8 * x1_76));
    st(0, 76, o0_76);
    const double x1_23 = ld(1, 23);
    const double x1_50 = ld(1, 50);
    const double x1_77 = ld(1, 77);
    double o0_23 = ((x0_0 * x1_23) + (x0_1 * x1_50) + (x0_2 * x1_77));
    st(0, 23, o0_23);
    double o0_50 = ((x0_3 * x1_23) + (x0_4 * x1_50) + (x0_5 * x1_77));
    st(0, 50, o0_50);
    double o0_77 = ((x0_6 * x1_23) + (x0_7 * x1_50) + (x0_8 * x1_77));
    st(0, 77, o0_77);
    const double x1_24 = ld(1, 24);
    const double x1_51 = ld(1, 51);
    const double x1_78 = ld(1, 78);
    double o0_24 = ((x0_0 * x1_24) + (x0_1 * x1_51) + (x0_2 * x1_78));
    st(0, 24, o0_24);
    double o0_51 = ((x0_3 * x1_24) + (x0_4 * x1_51) + (x0_5 * x1_78));
    st(0, 51, o0_51);
    double o0_78 = ((x0_6 * x1_24) + (x0_7 * x1_51) + (x0_8 * x1_78));
    st(0, 78, o0_78);
    const double x1_25 = ld(1, 25);
    const double x1_52 = ld(1, 52);
    const double x1_79 = ld(1, 79);
    double o0_25 = ((x0_0 * x1_25) + (x0_1 * x1_52) + (x0_2 * x1_79));
    st(0, 25, o0_25);
    double o0_52 = ((x0_3 * x1_25) + (x0_4 * x1_52) + (x0_5 * x1_79));
    st(0, 52, o0_52);
    double o0_79 = ((x0_6 * x1_25) + (x0_7 * x1_52) + (x0_8 * x1_79));
    st(0, 79, o0_79);
    const double x1_26 = ld(1, 26);
    const double x1_53 = ld(1, 53);
    const double x1_80 = ld(1, 80);
    double o0_26 = ((x0_0 * x1_26) + (x0_1 * x1_53) + (x0_2 * x1_80));
    st(0, 26, o0_26);
    double o0_53 = ((x0_3 * x1_26) + (x0_4 * x1_53) + (x0_5 * x1_80));
    st(0, 53, o0_53);
    double o0_80 = ((x0_6 * x1_26) + (x0_7 * x1_53) + (x0_8 * x1_80));
    st(0, 80, o0_80);
  }
};

// contract2: A_ijkl = C_j^n B_i^m E_mnkl (Sec. 5.1, eq:Contract2)
struct Gen_contract2 {
  static constexpr bool kStream = true;
  static constexpr int NF_IN = 3, NF_OUT = 1;
  static constexpr int fin[NF_IN] = {9, 9, 81};
  static constexpr int fout[NF_OUT] = {81};
  static constexpr int NIN = 99, NOUT = 81;
  template <class L, class S>
  __device__ static inline void stream(L&& ld, S&& st) {
    // A(i,j,k,l) = Sum(m, Sum(n, ((C(j,n) * B(i,m)) * E(m,n,k,l))))
    const double x1_0 = ld(1, 0);
    const double x0_0 = ld(0, 0);
    const double x2_0 = ld(2, 0);
    const double x0_1 = ld(0, 1);
    const double x2_9 = ld(2, 9);
    const double x0_2 = ld(0, 2);
    const double x2_18 = ld(2, 18);
    const double x1_1 = ld(1, 1);
    const double x2_27 = ld(2, 27);
    const double x2_36 = ld(2, 36);
    const double x2_45 = ld(2, 45);
    const double x1_2 = ld(1, 2);
    const double x2_54 = ld(2, 54);
    const double x2_63 = ld(2, 63);
    const double x2_72 = ld(2, 72);
    double o0_0 = ((x1_0 * ((x0_0 * x2_0) + (x0_1 * x2_9) + (x0_2 * x2_18))) + (x1_1 * ((x0_0 * x2_27) + (x0_1 * x2_36) + (x0_2 * x2_45))) + (x1_2 * ((x0_0 * x2_54) + (x0_1 * x2_63) + (x0_2 * x2_72))));
    st(0, 0, o0_0);
    const double x1_3 = ld(1, 3);
    const double x1_4 = ld(1, 4);
    const double x1_5 = ld(1, 5);
    double o0_27 = ((x1_3 * ((x0_0 * x2_0) + (x0_1 * x2_9) + (x0_2 * x2_18))) + (x1_4 * ((x0_0 * x2_27) + (x0_1 * x2_36) + (x0_2 * x2_45))) + (x1_5 * ((x0_0 * x2_54) + (x0_1 * x2_63) + (x0_2 * x2_72))));
    st(0, 27, o0_27);
    const double x1_6 = ld(1, 6);
    const double x1_7 = ld(1, 7);
    const double x1_8 = ld(1, 8);
    double o0_54 = ((x1_6 * ((x0_0 * x2_0) + (x0_1 * x2_9) + (x0_2 * x2_18))) + (x1_7 * ((x0_0 * x2_27) + (x0_1 * x2_36) + (x0_2 * x2_45))) + (x1_8 * ((x0_0 * x2_54) + (x0_1 * x2_63) + (x0_2 * x2_72))));
    st(0, 54, o0_54);
    const double x0_3 = ld(0, 3);
    const double x0_4 = ld(0, 4);
    const double x0_5 = ld(0, 5);
    double o0_9 = ((x1_0 * ((x0_3 * x2_0) + (x0_4 * x2_9) + (x0_5 * x2_18))) + (x1_1 * ((x0_3 * x2_27) + (x0_4 * x2_36) + (x0_5 * x2_45))) + (x1_2 * ((x0_3 * x2_54) + (x0_4 * x2_63) + (x0_5 * x2_72))));
    st(0, 9, o0_9);
    double o0_36 = ((x1_3 * ((x0_3 * x2_0) + (x0_4 * x2_9) + (x0_5 * x2_18))) + (x1_4 * ((x0_3 * x2_27) + (x0_4 * x2_36) + (x0_5 * x2_45))) + (x1_5 * ((x0_3 * x2_54) + (x0_4 * x2_63) + (x0_5 * x2_72))));
    st(0, 36, o0_36);
    double o0_63 = ((x1_6 * ((x0_3 * x2_0) + (x0_4 * x2_9) + (x0_5 * x2_18))) + (x1_7 * ((x0_3 * x2_27) + (x0_4 * x2_36) + (x0_5 * x2_45))) + (x1_8 * ((x0_3 * x2_54) + (x0_4 * x2_63) + (x0_5 * x2_72))));
    st(0, 63, o0_63);
    const double x0_6 = ld(0, 6);
    const double x0_7 = ld(0, 7);
    const double x0_8 = ld(0, 8);
    double o0_18 = ((x1_0 * ((x0_6 * x2_0) + (x0_7 * x2_9) + (x0_8 * x2_18))) + (x1_1 * ((x0_6 * x2_27) + (x0_7 * x2_36) + (x0_8 * x2_45))) + (x1_2 * ((x0_6 * x2_54) + (x0_7 * x2_63) + (x0_8 * x2_72))));
    st(0, 18, o0_18);
    double o0_45 = ((x1_3 * ((x0_6 * x2_0) + (x0_7 * x2_9) + (x0_8 * x2_18))) + (x1_4 * ((x0_6 * x2_27) + (x0_7 * x2_36) + (x0_8 * x2_45))) + (x1_5 * ((x0_6 * x2_54) + (x0_7 * x2_63) + (x0_8 * x2_72))));
    st(0, 45, o0_45);
    double o0_72 = ((x1_6 * ((x0_6 * x2_0) + (x0_7 * x2_9) + (x0_8 * x2_18))) + (x1_7 * ((x0_6 * x2_27) + (x0_7 * x2_36) + (x0_8 * x2_45))) + (x1_8 * ((x0_6 * x2_54) + (x0_7 * x2_63) + (x0_8 * x2_72))));
    st(0, 72, o0_72);
    const double x2_1 = ld(2, 1);
    const double x2_10 = ld(2, 10);
    const double x2_19 = ld(2, 19);
    const double x2_28 = ld(2, 28);
    const double x2_37 = ld(2, 37);
    const double x2_46 = ld(2, 46);
    const double x2_55 = ld(2, 55);
    const double x2_64 = ld(2, 64);
    const double x2_73 = ld(2, 73);
    double o0_1 = ((x1_0 * ((x0_0 * x2_1) + (x0_1 * x2_10) + (x0_2 * x2_19))) + (x1_1 * ((x0_0 * x2_28) + (x0_1 * x2_37) + (x0_2 * x2_46))) + (x1_2 * ((x0_0 * x2_55) + (x0_1 * x2_64) + (x0_2 * x2_73))));
    st(0, 1, o0_1);
    double o0_28 = ((x1_3 * ((x0_0 * x2_1) + (x0_1 * x2_10) + (x0_2 * x2_19))) + (x1_4 * ((x0_0 * x2_28) + (x0_1 * x2_37) + (x0_2 * x2_46))) + (x1_5 * ((x0_0 * x2_55) + (x0_1 * x2_64) + (x0_2 * x2_73))));
    st(0, 28, o0_28);
    double o0_55 = ((x1_6 * ((x0_0 * x2_1) + (x0_1 * x2_10) + (x0_2 * x2_19))) + (x1_7 * ((x0_0 * x2_28) + (x0_1 * x2_37) + (x0_2 * x2_46))) + (x1_8 * ((x0_0 * x2_55) + (x0_1 * x2_64) + (x0_2 * x2_73))));
    st(0, 55, o0_55);
    double o0_10 = ((x1_0 * ((x0_3 * x2_1) + (x0_4 * x2_10) + (x0_5 * x2_19))) + (x1_1 * ((x0_3 * x2_28) + (x0_4 * x2_37) + (x0_5 * x2_46))) + (x1_2 * ((x0_3 * x2_55) + (x0_4 * x2_64) + (x0_5 * x2_73))));
    st(0, 10, o0_10);
    double o0_37 = ((x1_3 * ((x0_3 * x2_1) + (x0_4 * x2_10) + (x0_5 * x2_19))) + (x1_4 * ((x0_3 * x2_28) + (x0_4 * x2_37) + (x0_5 * x2_46))) + (x1_5 * ((x0_3 * x2_55) + (x0_4 * x2_64) + (x0_5 * x2_73))));
    st(0, 37, o0_37);
    double o0_64 = ((x1_6 * ((x0_3 * x2_1) + (x0_4 * x2_10) + (x0_5 * x2_19))) + (x1_7 * ((x0_3 * x2_28) + (x0_4 * x2_37) + (x0_5 * x2_46))) + (x1_8 * ((x0_3 * x2_55) + (x0_4 * x2_64) + (x0_5 * x2_73))));
    st(0, 64, o0_64);
    double o0_19 = ((x1_0 * ((x0_6 * x2_1) + (x0_7 * x2_10) + (x0_8 * x2_19))) + (x1_1 * ((x0_6 * x2_28) + (x0_7 * x2_37) + (x0_8 * x2_46))) + (x1_2 * ((x0_6 * x2_55) + (x0_7 * x2_64) + (x0_8 * x2_73))));
    st(0, 19, o0_19);
    double o0_46 = ((x1_3 * ((x0_6 * x2_1) + (x0_7 * x2_10) + (x0_8 * x2_19))) + (x1_4 * ((x0_6 * x2_28) + (x0_7 * x2_37) + (x0_8 * x2_46))) + (x1_5 * ((x0_6 * x2_55) + (x0_7 * x2_64) + (x0_8 * x2_73))));
    st(0, 46, o0_46);
    double o0_73 = ((x1_6 * ((x0_6 * x2_1) + (x0_7 * x2_10) + (x0_8 * x2_19))) + (x1_7 * ((x0_6 * x2_28) + (x0_7 * x2_37) + (x0_8 * x2_46))) + (x1_8 * ((x0_6 * x2_55) + (x0_7 * x2_64) + (x0_8 * x2_73))));
    st(0, 73, o0_73);
    const double x2_2 = ld(2, 2);
    const double x2_11 = ld(2, 11);
    const double x2_20 = ld(2, 20);
    const double x2_29 = ld(2, 29);
    const double x2_38 = ld(2, 38);
    const double x2_47 = ld(2, 47);
    const double x2_56 = ld(2, 56);
    const double x2_65 = ld(2, 65);
    const double x2_74 = ld(2, 74);
    double o0_2 = ((x1_0 * ((x0_0 * x2_2) + (x0_1 * x2_11) + (x0_2 * x2_20))) + (x1_1 * ((x0_0 * x2_29) + (x0_1 * x2_38) + (x0_2 * x2_47))) + (x1_2 * ((x0_0 * x2_56) + (x0_1 * x2_65) + (x0_2 * x2_74))));
    st(0, 2, o0_2);
    double o0_29 = ((x1_3 * ((x0_0 * x2_2) + (x0_1 * x2_11) + (x0_2 * x2_20))) + (x1_4 * ((x0_0 * x2_29) + (x0_1 * x2_38) + (x0_2 * x2_47))) + (x1_5 * ((x0_0 * x2_56) + (x0_1 * x2_65) + (x0_2 * x2_74))));
    st(0, 29, o0_29);
    double o0_56 = ((x1_6 * ((x0_0 * x2_2) + (x0_1 * x2_11) + (x0_2 * x2_20))) + (x1_7 * ((x0_0 * x2_29) + (x0_1 * x2_38) + (x0_2 * x2_47))) + (x1_8 * ((x0_0 * x2_56) + (x0_1 * x2_65) + (x0_2 * x2_74))));
    st(0, 56, o0_56);
    double o0_11 = ((x1_0 * ((x0_3 * x2_2) + (x0_4 * x2_11) + (x0_5 * x2_20))) + (x1_1 * ((x0_3 * x2_29) + (x0_4 * x2_38) + (x0_5 * x2_47))) + (x1_2 * ((x0_3 * x2_56) + (x0_4 * x2_65) + (x0_5 * x2_74))));
    st(0, 11, o0_11);
    double o0_38 = ((x1_3 * ((x0_3 * x2_2) + (x0_4 * x2_11) + (x0_5 * x2_20))) + (x1_4 * ((x0_3 * x2_29) + (x0_4 * x2_38) + (x0_5 * x2_47))) + (x1_5 * ((x0_3 * x2_56) + (x0_4 * x2_65) + (x0_5 * x2_74))));
    st(0, 38, o0_38);
    double o0_65 = ((x1_6 * ((x0_3 * x2_2) + (x0_4 * x2_11) + (x0_5 * x2_20))) + (x1_7 * ((x0_3 * x2_29) + (x0_4 * x2_38) + (x0_5 * x2_47))) + (x1_8 * ((x0_3 * x2_56) + (x0_4 * x2_65) + (x0_5 * x2_74))));
    st(0, 65, o0_65);
    double o0_20 = ((x1_0 * ((x0_6 * x2_2) + (x0_7 * x2_11) + (x0_8 * x2_20))) + (x1_1 * ((x0_6 * x2_29) + (x0_7 * x2_38) + (x0_8 * x2_47))) + (x1_2 * ((x0_6 * x2_56) + (x0_7 * x2_65) + (x0_8 * x2_74))));
    st(0, 20, o0_20);
    double o0_47 = ((x1_3 * ((x0_6 * x2_2) + (x0_7 * x2_11) + (x0_8 * x2_20))) + (x1_4 * ((x0_6 * x2_29) + (x0_7 * x2_38) + (x0_8 * x2_47))) + (x1_5 * ((x0_6 * x2_56) + (x0_7 * x2_65) + (x0_8 * x2_74))));
    st(0, 47, o0_47);
    double o0_74 = ((x1_6 * ((x0_6 * x2_2) + (x0_7 * x2_11) + (x0_8 * x2_20))) + (x1_7 * ((x0_6 * x2_29) + (x0_7 * x2_38) + (x0_8 * x2_47))) + (x1_8 * ((x0_6 * x2_56) + (x0_7 * x2_65) + (x0_8 * x2_74))));
    st(0, 74, o0_74);
    __builtin_amdgcn_sched_barrier(0);
    const double x2_3 = ld(2, 3);
    const double x2_12 = ld(2, 12);
    const double x2_21 = ld(2, 21);
    const double x2_30 = ld(2, 30);
    const double x2_39 = ld(2, 39);
    const double x2_48 = ld(2, 48);
    const double x2_57 = ld(2, 57);
    const double x2_66 = ld(2, 66);
    const double x2_75 = ld(2, 75);
    double o0_3 = ((x1_0 * ((x0_0 * x2_3) + (x0_1 * x2_12) + (x0_2 * x2_21))) + (x1_1 * ((x0_0 * x2_30) + (x0_1 * x2_39) + (x0_2 * x2_48))) + (x1_2 * ((x0_0 * x2_57) + (x0_1 * x2_66) + (x0_2 * x2_75))));
    st(0, 3, o0_3);
    double o0_30 = ((x1_3 * ((x0_0 * x2_3) + (x0_1 * x2_12) + (x0_2 * x2_21))) + (x1_4 * ((x0_0 * x2_30) + (x0_1 * x2_39) + (x0_2 * x2_48))) + (x1_5 * ((x0_0 * x2_57) + (x0_1 * x2_66) + (x0_2 * x2_75))));
    st(0, 30, o0_30);
    double o0_57 = ((x1_6 * ((x0_0 * x2_3) + (x0_1 * x2_12) + (x0_2 * x2_21))) + (x1_7 * ((x0_0 * x2_30) + (x0_1 * x2_39) + (x0_2 * x2_48))) + (x1_8 * ((x0_0 * x2_57) + (x0_1 * x2_66) + (x0_2 * x2_75))));
    st(0, 57, o0_57);
    double o0_12 = ((x1_0 * ((x0_3 * x2_3) + (x0_4 * x2_12) + (x0_5 * x2_21))) + (x1_1 * ((x0_3 * x2_30) + (x0_4 * x2_39) + (x0_5 * x2_48))) + (x1_2 * ((x0_3 * x2_57) + (x0_4 * x2_66) + (x0_5 * x2_75))));
    st(0, 12, o0_12);
    double o0_39 = ((x1_3 * ((x0_3 * x2_3) + (x0_4 * x2_12) + (x0_5 * x2_21))) + (x1_4 * ((x0_3 * x2_30) + (x0_4 * x2_39) + (x0_5 * x2_48))) + (x1_5 * ((x0_3 * x2_57) + (x0_4 * x2_66) + (x0_5 * x2_75))));
    st(0, 39, o0_39);
    double o0_66 = ((x1_6 * ((x0_3 * x2_3) + (x0_4 * x2_12) + (x0_5 * x2_21))) + (x1_7 * ((x0_3 * x2_30) + (x0_4 * x2_39) + (x0_5 * x2_48))) + (x1_8 * ((x0_3 * x2_57) + (x0_4 * x2_66) + (x0_5 * x2_75))));
    st(0, 66, o0_66);
    double o0_21 = ((x1_0 * ((x0_6 * x2_3) + (x0_7 * x2_12) + (x0_8 * x2_21))) + (x1_1 * ((x0_6 * x2_30) + (x0_7 * x2_39) + (x0_8 * x2_48))) + (x1_2 * ((x0_6 * x2_57) + (x0_7 * x2_66) + (x0_8 * x2_75))));
    st(0, 21, o0_21);
    double o0_48 = ((x1_3 * ((x0_6 * x2_3) + (x0_7 * x2_12) + (x0_8 * x2_21))) + (x1_4 * ((x0_6 * x2_30) + (x0_7 * x2_39) + (x0_8 * x2_48))) + (x1_5 * ((x0_6 * x2_57) + (x0_7 * x2_66) + (x0_8 * x2_75))));
    st(0, 48, o0_48);
    double o0_75 = ((x1_6 * ((x0_6 * x2_3) + (x0_7 * x2_12) + (x0_8 * x2_21))) + (x1_7 * ((x0_6 * x2_30) + (x0_7 * x2_39) + (x0_8 * x2_48))) + (x1_8 * ((x0_6 * x2_57) + (x0_7 * x2_66) + (x0_8 * x2_75))));
    st(0, 75, o0_75);
    const double x2_4 = ld(2, 4);
    const double x2_13 = ld(2, 13);
    const double x2_22 = ld(2, 22);
    const double x2_31 = ld(2, 31);
    const double x2_40 = ld(2, 40);
    const double x2_49 = ld(2, 49);
    const double x2_58 = ld(2, 58);
    const double x2_67 = ld(2, 67);
    const double x2_76 = ld(2, 76);
    double o0_4 = ((x1_0 * ((x0_0 * x2_4) + (x0_1 * x2_13) + (x0_2 * x2_22))) + (x1_1 * ((x0_0 * x2_31) + (x0_1 * x2_40) + (x0_2 * x2_49))) + (x1_2 * ((x0_0 * x2_58) + (x0_1 * x2_67) + (x0_2 * x2_76))));
    st(0, 4, o0_4);
    double o0_31 = ((x1_3 * ((x0_0 * x2_4) + (x0_1 * x2_13) + (x0_2 * x2_22))) + (x1_4 * ((x0_0 * x2_31) + (x0_1 * x2_40) + (x0_2 * x2_49))) + (x1_5 * ((x0_0 * x2_58) + (x0_1 * x2_67) + (x0_2 * x2_76))));
    st(0, 31, o0_31);
    double o0_58 = ((x1_6 * ((x0_0 * x2_4) + (x0_1 * x2_13) + (x0_2 * x2_22))) + (x1_7 * ((x0_0 * x2_31) + (x0_1 * x2_40) + (x0_2 * x2_49))) + (x1_8 * ((x0_0 * x2_58) + (x0_1 * x2_67) + (x0_2 * x2_76))));
    st(0, 58, o0_58);
    double o0_13 = ((x1_0 * ((x0_3 * x2_4) + (x0_4 * x2_13) + (x0_5 * x2_22))) + (x1_1 * ((x0_3 * x2_31) + (x0_4 * x2_40) + (x0_5 * x2_49))) + (x1_2 * ((x0_3 * x2_58) + (x0_4 * x2_67) + (x0_5 * x2_76))));
    st(0, 13, o0_13);
    double o0_40 = ((x1_3 * ((x0_3 * x2_4) + (x0_4 * x2_13) + (x0_5 * x2_22))) + (x1_4 * ((x0_3 * x2_31) + (x0_4 * x2_40) + (x0_5 * x2_49))) + (x1_5 * ((x0_3 * x2_58) + (x0_4 * x2_67) + (x0_5 * x2_76))));
    st(0, 40, o0_40);
    double o0_67 = ((x1_6 * ((x0_3 * x2_4) + (x0_4 * x2_13) + (x0_5 * x2_22))) + (x1_7 * ((x0_3 * x2_31) + (x0_4 * x2_40) + (x0_5 * x2_49))) + (x1_8 * ((x0_3 * x2_58) + (x0_4 * x2_67) + (x0_5 * x2_76))));
    st(0, 67, o0_67);
    double o0_22 = ((x1_0 * ((x0_6 * x2_4) + (x0_7 * x2_13) + (x0_8 * x2_22))) + (x1_1 * ((x0_6 * x2_31) + (x0_7 * x2_40) + (x0_8 * x2_49))) + (x1_2 * ((x0_6 * x2_58) + (x0_7 * x2_67) + (x0_8 * x2_76))));
    st(0, 22, o0_22);
    double o0_49 = ((x1_3 * ((x0_6 * x2_4) + (x0_7 * x2_13) + (x0_8 * x2_22))) + (x1_4 * ((x0_6 * x2_31) + (x0_7 * x2_40) + (x0_8 * x2_49))) + (x1_5 * ((x0_6 * x2_58) + (x0_7 * x2_67) + (x0_8 * x2_76))));
    st(0, 49, o0_49);
    double o0_76 = ((x1_6 * ((x0_6 * x2_4) + (x0_7 * x2_13) + (x0_8 * x2_22))) + (x1_7 * ((x0_6 * x2_31) + (x0_7 * x2_40) + (x0_8 * x2_49))) + (x1_8 * ((x0_6 * x2_58) + (x0_7 * x2_67) + (x0_8 * x2_76))));
    st(0, 76, o0_76);
    const double x2_5 = ld(2, 5);
    const double x2_14 = ld(2, 14);
    const double x2_23 = ld(2, 23);
    const double x2_32 = ld(2, 32);
    const double x2_41 = ld(2, 41);
    const double x2_50 = ld(2, 50);
    const double x2_59 = ld(2, 59);
    const double x2_68 = ld(2, 68);
    const double x2_77 = ld(2, 77);
    double o0_5 = ((x1_0 * ((x0_0 * x2_5) + (x0_1 * x2_14) + (x0_2 * x2_23))) + (x1_1 * ((x0_0 * x2_32) + (x0_1 * x2_41) + (x0_2 * x2_50))) + (x1_2 * ((x0_0 * x2_59) + (x0_1 * x2_68) + (x0_2 * x2_77))));
    st(0, 5, o0_5);
    double o0_32 = ((x1_3 * ((x0_0 * x2_5) + (x0_1 * x2_14) + (x0_2 * x2_23))) + (x1_4 * ((x0_0 * x2_32) + (x0_1 * x2_41) + (x0_2 * x2_50))) + (x1_5 * ((x0_0 * x2_59) + (x0_1 * x2_68) + (x0_2 * x2_77))));
    st(0, 32, o0_32);
    double o0_59 = ((x1_6 * ((x0_0 * x2_5) + (x0_1 * x2_14) + (x0_2 * x2_23))) + (x1_7 * ((x0_0 * x2_32) + (x0_1 * x2_41) + (x0_2 * x2_50))) + (x1_8 * ((x0_0 * x2_59) + (x0_1 * x2_68) + (x0_2 * x2_77))));
    st(0, 59, o0_59);
    double o0_14 = ((x1_0 * ((x0_3 * x2_5) + (x0_4 * x2_14) + (x0_5 * x2_23))) + (x1_1 * ((x0_3 * x2_32) + (x0_4 * x2_41) + (x0_5 * x2_50))) + (x1_2 * ((x0_3 * x2_59) + (x0_4 * x2_68) + (x0_5 * x2_77))));
    st(0, 14, o0_14);
    double o0_41 = ((x1_3 * ((x0_3 * x2_5) + (x0_4 * x2_14) + (x0_5 * x2_23))) + (x1_4 * ((x0_3 * x2_32) + (x0_4 * x2_41) + (x0_5 * x2_50))) + (x1_5 * ((x0_3 * x2_59) + (x0_4 * x2_68) + (x0_5 * x2_77))));
    st(0, 41, o0_41);
    double o0_68 = ((x1_6 * ((x0_3 * x2_5) + (x0_4 * x2_14) + (x0_5 * x2_23))) + (x1_7 * ((x0_3 * x2_32) + (x0_4 * x2_41) + (x0_5 * x2_50))) + (x1_8 * ((x0_3 * x2_59) + (x0_4 * x2_68) + (x0_5 * x2_77))));
    st(0, 68, o0_68);
    double o0_23 = ((x1_0 * ((x0_6 * x2_5) + (x0_7 * x2_14) + (x0_8 * x2_23))) + (x1_1 * ((x0_6 * x2_32) + (x0_7 * x2_41) + (x0_8 * x2_50))) + (x1_2 * ((x0_6 * x2_59) + (x0_7 * x2_68) + (x0_8 * x2_77))));
    st(0, 23, o0_23);
    double o0_50 = ((x1_3 * ((x0_6 * x2_5) + (x0_7 * x2_14) + (x0_8 * x2_23))) + (x1_4 * ((x0_6 * x2_32) + (x0_7 * x2_41) + (x0_8 * x2_50))) + (x1_5 * ((x0_6 * x2_59) + (x0_7 * x2_68) + (x0_8 * x2_77))));
    st(0, 50, o0_50);
    double o0_77 = ((x1_6 * ((x0_6 * x2_5) + (x0_7 * x2_14) + (x0_8 * x2_23))) + (x1_7 * ((x0_6 * x2_32) + (x0_7 * x2_41) + (x0_8 * x2_50))) + (x1_8 * ((x0_6 * x2_59) + (x0_7 * x2_68) + (x0_8 * x2_77))));
    st(0, 77, o0_77);
    __builtin_amdgcn_sched_barrier(0);
    const double x2_6 = ld(2, 6);
    const double x2_15 = ld(2, 15);
    const double x2_24 = ld(2, 24);
    const double x2_33 = ld(2, 33);
    const double x2_42 = ld(2, 42);
    const double x2_51 = ld(2, 51);
    const double x2_60 = ld(2, 60);
    const double x2_69 = ld(2, 69);
    const double x2_78 = ld(2, 78);
    double o0_6 = ((x1_0 * ((x0_0 * x2_6) + (x0_1 * x2_15) + (x0_2 * x2_24))) + (x1_1 * ((x0_0 * x2_33) + (x0_1 * x2_42) + (x0_2 * x2_51))) + (x1_2 * ((x0_0 * x2_60) + (x0_1 * x2_69) + (x0_2 * x2_78))));
    st(0, 6, o0_6);
    double o0_33 = ((x1_3 * ((x0_0 * x2_6) + (x0_1 * x2_15) + (x0_2 * x2_24))) + (x1_4 * ((x0_0 * x2_33) + (x0_1 * x2_42) + (x0_2 * x2_51))) + (x1_5 * ((x0_0 * x2_60) + (x0_1 * x2_69) + (x0_2 * x2_78))));
    st(0, 33, o0_33);
    double o0_60 = ((x1_6 * ((x0_0 * x2_6) + (x0_1 * x2_15) + (x0_2 * x2_24))) + (x1_7 * ((x0_0 * x2_33) + (x0_1 * x2_42) + (x0_2 * x2_51))) + (x1_8 * ((x0_0 * x2_60) + (x0_1 * x2_69) + (x0_2 * x2_78))));
    st(0, 60, o0_60);
    double o0_15 = ((x1_0 * ((x0_3 * x2_6) + (x0_4 * x2_15) + (x0_5 * x2_24))) + (x1_1 * ((x0_3 * x2_33) + (x0_4 * x2_42) + (x0_5 * x2_51))) + (x1_2 * ((x0_3 * x2_60) + (x0_4 * x2_69) + (x0_5 * x2_78))));
    st(0, 15, o0_15);
    double o0_42 = ((x1_3 * ((x0_3 * x2_6) + (x0_4 * x2_15) + (x0_5 * x2_24))) + (x1_4 * ((x0_3 * x2_33) + (x0_4 * x2_42) + (x0_5 * x2_51))) + (x1_5 * ((x0_3 * x2_60) + (x0_4 * x2_69) + (x0_5 * x2_78))));
    st(0, 42, o0_42);
    double o0_69 = ((x1_6 * ((x0_3 * x2_6) + (x0_4 * x2_15) + (x0_5 * x2_24))) + (x1_7 * ((x0_3 * x2_33) + (x0_4 * x2_42) + (x0_5 * x2_51))) + (x1_8 * ((x0_3 * x2_60) + (x0_4 * x2_69) + (x0_5 * x2_78))));
    st(0, 69, o0_69);
    double o0_24 = ((x1_0 * ((x0_6 * x2_6) + (x0_7 * x2_15) + (x0_8 * x2_24))) + (x1_1 * ((x0_6 * x2_33) + (x0_7 * x2_42) + (x0_8 * x2_51))) + (x1_2 * ((x0_6 * x2_60) + (x0_7 * x2_69) + (x0_8 * x2_78))));
    st(0, 24, o0_24);
    double o0_51 = ((x1_3 * ((x0_6 * x2_6) + (x0_7 * x2_15) + (x0_8 * x2_24))) + (x1_4 * ((x0_6 * x2_33) + (x0_7 * x2_42) + (x0_8 * x2_51))) + (x1_5 * ((x0_6 * x2_60) + (x0_7 * x2_69) + (x0_8 * x2_78))));
    st(0, 51, o0_51);
    double o0_78 = ((x1_6 * ((x0_6 * x2_6) + (x0_7 * x2_15) + (x0_8 * x2_24))) + (x1_7 * ((x0_6 * x2_33) + (x0_7 * x2_42) + (x0_8 * x2_51))) + (x1_8 * ((x0_6 * x2_60) + (x0_7 * x2_69) + (x0_8 * x2_78))));
    st(0, 78, o0_78);
    const double x2_7 = ld(2, 7);
    const double x2_16 = ld(2, 16);
    const double x2_25 = ld(2, 25);
    const double x2_34 = ld(2, 34);
    const double x2_43 = ld(2, 43);
    const double x2_52 = ld(2, 52);
    const double x2_61 = ld(2, 61);
    const double x2_70 = ld(2, 70);
    const double x2_79 = ld(2, 79);
    double o0_7 = ((x1_0 * ((x0_0 * x2_7) + (x0_1 * x2_16) + (x0_2 * x2_25))) + (x1_1 * ((x0_0 * x2_34) + (x0_1 * x2_43) + (x0_2 * x2_52))) + (x1_2 * ((x0_0 * x2_61) + (x0_1 * x2_70) + (x0_2 * x2_79))));
    st(0, 7, o0_7);
    double o0_34 = ((x1_3 * ((x0_0 * x2_7) + (x0_1 * x2_16) + (x0_2 * x2_25))) + (x1_4 * ((x0_0 * x2_34) + (x0_1 * x2_43) + (x0_2 * x2_52))) + (x1_5 * ((x0_0 * x2_61) + (x0_1 * x2_70) + (x0_2 * x2_79))));
    st(0, 34, o0_34);
    double o0_61 = ((x1_6 * ((x0_0 * x2_7) + (x0_1 * x2_16) + (x0_2 * x2_25))) + (x1_7 * ((x0_0 * x2_34) + (x0_1 * x2_43) + (x0_2 * x2_52))) + (x1_8 * ((x0_0 * x2_61) + (x0_1 * x2_70) + (x0_2 * x2_79))));
    st(0, 61, o0_61);
    double o0_16 = ((x1_0 * ((x0_3 * x2_7) + (x0_4 * x2_16) + (x0_5 * x2_25))) + (x1_1 * ((x0_3 * x2_34) + (x0_4 * x2_43) + (x0_5 * x2_52))) + (x1_2 * ((x0_3 * x2_61) + (x0_4 * x2_70) + (x0_5 * x2_79))));
    st(0, 16, o0_16);
    double o0_43 = ((x1_3 * ((x0_3 * x2_7) + (x0_4 * x2_16) + (x0_5 * x2_25))) + (x1_4 * ((x0_3 * x2_34) + (x0_4 * x2_43) + (x0_5 * x2_52))) + (x1_5 * ((x0_3 * x2_61) + (x0_4 * x2_70) + (x0_5 * x2_79))));
    st(0, 43, o0_43);
    double o0_70 = ((x1_6 * ((x0_3 * x2_7) + (x0_4 * x2_16) + (x0_5 * x2_25))) + (x1_7 * ((x0_3 * x2_34) + (x0_4 * x2_43) + (x0_5 * x2_52))) + (x1_8 * ((x0_3 * x2_61) + (x0_4 * x2_70) + (x0_5 * x2_79))));
    st(0, 70, o0_70);
    double o0_25 = ((x1_0 * ((x0_6 * x2_7) + (x0_7 * x2_16) + (x0_8 * x2_25))) + (x1_1 * ((x0_6 * x2_34) + (x0_7 * x2_43) + (x0_8 * x2_52))) + (x1_2 * ((x0_6 * x2_61) + (x0_7 * x2_70) + (x0_8 * x2_79))));
    st(0, 25, o0_25);
    double o0_52 = ((x1_3 * ((x0_6 * x2_7) + (x0_7 * x2_16) + (x0_8 * x2_25))) + (x1_4 * ((x0_6 * x2_34) + (x0_7 * x2_43) + (x0_8 * x2_52))) + (x1_5 * ((x0_6 * x2_61) + (x0_7 * x2_70) + (x0_8 * x2_79))));
    st(0, 52, o0_52);
    double o0_79 = ((x1_6 * ((x0_6 * x2_7) + (x0_7 * x2_16) + (x0_8 * x2_25))) + (x1_7 * ((x0_6 * x2_34) + (x0_7 * x2_43) + (x0_8 * x2_52))) + (x1_8 * ((x0_6 * x2_61) + (x0_7 * x2_70) + (x0_8 * x2_79))));
    st(0, 79, o0_79);
    const double x2_8 = ld(2, 8);
    const double x2_17 = ld(2, 17);
    const double x2_26 = ld(2, 26);
    const double x2_35 = ld(2, 35);
    const double x2_44 = ld(2, 44);
    const double x2_53 = ld(2, 53);
    const double x2_62 = ld(2, 62);
    const double x2_71 = ld(2, 71);
    const double x2_80 = ld(2, 80);
    double o0_8 = ((x1_0 * ((x0_0 * x2_8) + (x0_1 * x2_17) + (x0_2 * x2_26))) + (x1_1 * ((x0_0 * x2_35) + (x0_1 * x2_44) + (x0_2 * x2_53))) + (x1_2 * ((x0_0 * x2_62) + (x0_1 * x2_71) + (x0_2 * x2_80))));
    st(0, 8, o0_8);
    double o0_35 = ((x1_3 * ((x0_0 * x2_8) + (x0_1 * x2_17) + (x0_2 * x2_26))) + (x1_4 * ((x0_0 * x2_35) + (x0_1 * x2_44) + (x0_2 * x2_53))) + (x1_5 * ((x0_0 * x2_62) + (x0_1 * x2_71) + (x0_2 * x2_80))));
    st(0, 35, o0_35);
    double o0_62 = ((x1_6 * ((x0_0 * x2_8) + (x0_1 * x2_17) + (x0_2 * x2_26))) + (x1_7 * ((x0_0 * x2_35) + (x0_1 * x2_44) + (x0_2 * x2_53))) + (x1_8 * ((x0_0 * x2_62) + (x0_1 * x2_71) + (x0_2 * x2_80))));
    st(0, 62, o0_62);
    double o0_17 = ((x1_0 * ((x0_3 * x2_8) + (x0_4 * x2_17) + (x0_5 * x2_26))) + (x1_1 * ((x0_3 * x2_35) + (x0_4 * x2_44) + (x0_5 * x2_53))) + (x1_2 * ((x0_3 * x2_62) + (x0_4 * x2_71) + (x0_5 * x2_80))));
    st(0, 17, o0_17);
    double o0_44 = ((x1_3 * ((x0_3 * x2_8) + (x0_4 * x2_17) + (x0_5 * x2_26))) + (x1_4 * ((x0_3 * x2_35) + (x0_4 * x2_44) + (x0_5 * x2_53))) + (x1_5 * ((x0_3 * x2_62) + (x0_4 * x2_71) + (x0_5 * x2_80))));
    st(0, 44, o0_44);
    double o0_71 = ((x1_6 * ((x0_3 * x2_8) + (x0_4 * x2_17) + (x0_5 * x2_26))) + (x1_7 * ((x0_3 * x2_35) + (x0_4 * x2_44) + (x0_5 * x2_53))) + (x1_8 * ((x0_3 * x2_62) + (x0_4 * x2_71) + (x0_5 * x2_80))));
    st(0, 71, o0_71);
    double o0_26 = ((x1_0 * ((x0_6 * x2_8) + (x0_7 * x2_17) + (x0_8 * x2_26))) + (x1_1 * ((x0_6 * x2_35) + (x0_7 * x2_44) + (x0_8 * x2_53))) + (x1_2 * ((x0_6 * x2_62) + (x0_7 * x2_71) + (x0_8 * x2_80))));
    st(0, 26, o0_26);
    double o0_53 = ((x1_3 * ((x0_6 * x2_8) + (x0_7 * x2_17) + (x0_8 * x2_26))) + (x1_4 * ((x0_6 * x2_35) + (x0_7 * x2_44) + (x0_8 * x2_53))) + (x1_5 * ((x0_6 * x2_62) + (x0_7 * x2_71) + (x0_8 * x2_80))));
    st(0, 53, o0_53);
    double o0_80 = ((x1_6 * ((x0_6 * x2_8) + (x0_7 * x2_17) + (x0_8 * x2_26))) + (x1_7 * ((x0_6 * x2_35) + (x0_7 * x2_44) + (x0_8 * x2_53))) + (x1_8 * ((x0_6 * x2_62) + (x0_7 * x2_71) + (x0_8 * x2_80))));
    st(0, 80, o0_80);
  }
};

// contract3: A_ijkl = D_k^o C_j^n B_i^m E_mnol (Sec. 5.1, eq:Contract3)
struct Gen_contract3 {
  static constexpr bool kStream = true;
  static constexpr int kMaxBlock = 256;  // more than 100 inputs
  static constexpr int NF_IN = 4, NF_OUT = 1;
  static constexpr int fin[NF_IN] = {9, 9, 9, 81};
  static constexpr int fout[NF_OUT] = {81};
  static constexpr int NIN = 108, NOUT = 81;
  template <class L, class S>
  __device__ static inline void stream(L&& ld, S&& st) {
    double t_T[81];
    double t_M[81];
    // T(i,n,o,l) = Sum(m, (B(i,m) * E(m,n,o,l)))
    // M(i,j,o,l) = Sum(n, (C(j,n) * T(i,n,o,l)))
    // A(i,j,k,l) = Sum(o, (D(k,o) * M(i,j,o,l)))
    // slice by slice in l
    const double x2_0 = ld(2, 0);
    const double x3_0 = ld(3, 0);
    const double x2_1 = ld(2, 1);
    const double x3_27 = ld(3, 27);
    const double x2_2 = ld(2, 2);
    const double x3_54 = ld(3, 54);
    t_T[0] = ((x2_0 * x3_0) + (x2_1 * x3_27) + (x2_2 * x3_54));
    const double x2_3 = ld(2, 3);
    const double x2_4 = ld(2, 4);
    const double x2_5 = ld(2, 5);
    t_T[27] = ((x2_3 * x3_0) + (x2_4 * x3_27) + (x2_5 * x3_54));
    const double x2_6 = ld(2, 6);
    const double x2_7 = ld(2, 7);
    const double x2_8 = ld(2, 8);
    t_T[54] = ((x2_6 * x3_0) + (x2_7 * x3_27) + (x2_8 * x3_54));
    const double x3_3 = ld(3, 3);
    const double x3_30 = ld(3, 30);
    const double x3_57 = ld(3, 57);
    t_T[3] = ((x2_0 * x3_3) + (x2_1 * x3_30) + (x2_2 * x3_57));
    t_T[30] = ((x2_3 * x3_3) + (x2_4 * x3_30) + (x2_5 * x3_57));
    t_T[57] = ((x2_6 * x3_3) + (x2_7 * x3_30) + (x2_8 * x3_57));
    const double x3_6 = ld(3, 6);
    const double x3_33 = ld(3, 33);
    const double x3_60 = ld(3, 60);
    t_T[6] = ((x2_0 * x3_6) + (x2_1 * x3_33) + (x2_2 * x3_60));
    t_T[33] = ((x2_3 * x3_6) + (x2_4 * x3_33) + (x2_5 * x3_60));
    t_T[60] = ((x2_6 * x3_6) + (x2_7 * x3_33) + (x2_8 * x3_60));
    __builtin_amdgcn_sched_barrier(0);
    const double x3_9 = ld(3, 9);
    const double x3_36 = ld(3, 36);
    const double x3_63 = ld(3, 63);
    t_T[9] = ((x2_0 * x3_9) + (x2_1 * x3_36) + (x2_2 * x3_63));
    t_T[36] = ((x2_3 * x3_9) + (x2_4 * x3_36) + (x2_5 * x3_63));
    t_T[63] = ((x2_6 * x3_9) + (x2_7 * x3_36) + (x2_8 * x3_63));
    const double x3_12 = ld(3, 12);
    const double x3_39 = ld(3, 39);
    const double x3_66 = ld(3, 66);
    t_T[12] = ((x2_0 * x3_12) + (x2_1 * x3_39) + (x2_2 * x3_66));
    t_T[39] = ((x2_3 * x3_12) + (x2_4 * x3_39) + (x2_5 * x3_66));
    t_T[66] = ((x2_6 * x3_12) + (x2_7 * x3_39) + (x2_8 * x3_66));
    const double x3_15 = ld(3, 15);
    const double x3_42 = ld(3, 42);
    const double x3_69 = ld(3, 69);
    t_T[15] = ((x2_0 * x3_15) + (x2_1 * x3_42) + (x2_2 * x3_69));
    t_T[42] = ((x2_3 * x3_15) + (x2_4 * x3_42) + (x2_5 * x3_69));
    t_T[69] = ((x2_6 * x3_15) + (x2_7 * x3_42) + (x2_8 * x3_69));
    __builtin_amdgcn_sched_barrier(0);
    const double x3_18 = ld(3, 18);
    const double x3_45 = ld(3, 45);
    const double x3_72 = ld(3, 72);
    t_T[18] = ((x2_0 * x3_18) + (x2_1 * x3_45) + (x2_2 * x3_72));
    t_T[45] = ((x2_3 * x3_18) + (x2_4 * x3_45) + (x2_5 * x3_72));
    t_T[72] = ((x2_6 * x3_18) + (x2_7 * x3_45) + (x2_8 * x3_72));
    const double x3_21 = ld(3, 21);
    const double x3_48 = ld(3, 48);
    const double x3_75 = ld(3, 75);
    t_T[21] = ((x2_0 * x3_21) + (x2_1 * x3_48) + (x2_2 * x3_75));
    t_T[48] = ((x2_3 * x3_21) + (x2_4 * x3_48) + (x2_5 * x3_75));
    t_T[75] = ((x2_6 * x3_21) + (x2_7 * x3_48) + (x2_8 * x3_75));
    const double x3_24 = ld(3, 24);
    const double x3_51 = ld(3, 51);
    const double x3_78 = ld(3, 78);
    t_T[24] = ((x2_0 * x3_24) + (x2_1 * x3_51) + (x2_2 * x3_78));
    t_T[51] = ((x2_3 * x3_24) + (x2_4 * x3_51) + (x2_5 * x3_78));
    t_T[78] = ((x2_6 * x3_24) + (x2_7 * x3_51) + (x2_8 * x3_78));
    const double x1_0 = ld(1, 0);
    const double x1_1 = ld(1, 1);
    const double x1_2 = ld(1, 2);
    t_M[0] = ((x1_0 * t_T[0]) + (x1_1 * t_T[9]) + (x1_2 * t_T[18]));
    const double x1_3 = ld(1, 3);
    const double x1_4 = ld(1, 4);
    const double x1_5 = ld(1, 5);
    t_M[9] = ((x1_3 * t_T[0]) + (x1_4 * t_T[9]) + (x1_5 * t_T[18]));
    const double x1_6 = ld(1, 6);
    const double x1_7 = ld(1, 7);
    const double x1_8 = ld(1, 8);
    t_M[18] = ((x1_6 * t_T[0]) + (x1_7 * t_T[9]) + (x1_8 * t_T[18]));
    t_M[3] = ((x1_0 * t_T[3]) + (x1_1 * t_T[12]) + (x1_2 * t_T[21]));
    t_M[12] = ((x1_3 * t_T[3]) + (x1_4 * t_T[12]) + (x1_5 * t_T[21]));
    t_M[21] = ((x1_6 * t_T[3]) + (x1_7 * t_T[12]) + (x1_8 * t_T[21]));
    t_M[6] = ((x1_0 * t_T[6]) + (x1_1 * t_T[15]) + (x1_2 * t_T[24]));
    t_M[15] = ((x1_3 * t_T[6]) + (x1_4 * t_T[15]) + (x1_5 * t_T[24]));
    t_M[24] = ((x1_6 * t_T[6]) + (x1_7 * t_T[15]) + (x1_8 * t_T[24]));
    __builtin_amdgcn_sched_barrier(0);
    t_M[27] = ((x1_0 * t_T[27]) + (x1_1 * t_T[36]) + (x1_2 * t_T[45]));
    t_M[36] = ((x1_3 * t_T[27]) + (x1_4 * t_T[36]) + (x1_5 * t_T[45]));
    t_M[45] = ((x1_6 * t_T[27]) + (x1_7 * t_T[36]) + (x1_8 * t_T[45]));
    t_M[30] = ((x1_0 * t_T[30]) + (x1_1 * t_T[39]) + (x1_2 * t_T[48]));
    t_M[39] = ((x1_3 * t_T[30]) + (x1_4 * t_T[39]) + (x1_5 * t_T[48]));
    t_M[48] = ((x1_6 * t_T[30]) + (x1_7 * t_T[39]) + (x1_8 * t_T[48]));
    t_M[33] = ((x1_0 * t_T[33]) + (x1_1 * t_T[42]) + (x1_2 * t_T[51]));
    t_M[42] = ((x1_3 * t_T[33]) + (x1_4 * t_T[42]) + (x1_5 * t_T[51]));
    t_M[51] = ((x1_6 * t_T[33]) + (x1_7 * t_T[42]) + (x1_8 * t_T[51]));
    __builtin_amdgcn_sched_barrier(0);
    t_M[54] = ((x1_0 * t_T[54]) + (x1_1 * t_T[63]) + (x1_2 * t_T[72]));
    t_M[63] = ((x1_3 * t_T[54]) + (x1_4 * t_T[63]) + (x1_5 * t_T[72]));
    t_M[72] = ((x1_6 * t_T[54]) + (x1_7 * t_T[63]) + (x1_8 * t_T[72]));
    t_M[57] = ((x1_0 * t_T[57]) + (x1_1 * t_T[66]) + (x1_2 * t_T[75]));
    t_M[66] = ((x1_3 * t_T[57]) + (x1_4 * t_T[66]) + (x1_5 * t_T[75]));
    t_M[75] = ((x1_6 * t_T[57]) + (x1_7 * t_T[66]) + (x1_8 * t_T[75]));
    t_M[60] = ((x1_0 * t_T[60]) + (x1_1 * t_T[69]) + (x1_2 * t_T[78]));
    t_M[69] = ((x1_3 * t_T[60]) + (x1_4 * t_T[69]) + (x1_5 * t_T[78]));
    t_M[78] = ((x1_6 * t_T[60]) + (x1_7 * t_T[69]) + (x1_8 * t_T[78]));
    const double x0_0 = ld(0, 0);
    const double x0_1 = ld(0, 1);
    const double x0_2 = ld(0, 2);
    double o0_0 = ((x0_0 * t_M[0]) + (x0_1 * t_M[3]) + (x0_2 * t_M[6]));
    st(0, 0, o0_0);
    const double x0_3 = ld(0, 3);
    const double x0_4 = ld(0, 4);
    const double x0_5 = ld(0, 5);
    double o0_3 = ((x0_3 * t_M[0]) + (x0_4 * t_M[3]) + (x0_5 * t_M[6]));
    st(0, 3, o0_3);
    const double x0_6 = ld(0, 6);
    const double x0_7 = ld(0, 7);
    const double x0_8 = ld(0, 8);
    double o0_6 = ((x0_6 * t_M[0]) + (x0_7 * t_M[3]) + (x0_8 * t_M[6]));
    st(0, 6, o0_6);
    double o0_9 = ((x0_0 * t_M[9]) + (x0_1 * t_M[12]) + (x0_2 * t_M[15]));
    st(0, 9, o0_9);
    double o0_12 = ((x0_3 * t_M[9]) + (x0_4 * t_M[12]) + (x0_5 * t_M[15]));
    st(0, 12, o0_12);
    double o0_15 = ((x0_6 * t_M[9]) + (x0_7 * t_M[12]) + (x0_8 * t_M[15]));
    st(0, 15, o0_15);
    double o0_18 = ((x0_0 * t_M[18]) + (x0_1 * t_M[21]) + (x0_2 * t_M[24]));
    st(0, 18, o0_18);
    double o0_21 = ((x0_3 * t_M[18]) + (x0_4 * t_M[21]) + (x0_5 * t_M[24]));
    st(0, 21, o0_21);
    double o0_24 = ((x0_6 * t_M[18]) + (x0_7 * t_M[21]) + (x0_8 * t_M[24]));
    st(0, 24, o0_24);
    __builtin_amdgcn_sched_barrier(0);
    double o0_27 = ((x0_0 * t_M[27]) + (x0_1 * t_M[30]) + (x0_2 * t_M[33]));
    st(0, 27, o0_27);
    double o0_30 = ((x0_3 * t_M[27]) + (x0_4 * t_M[30]) + (x0_5 * t_M[33]));
    st(0, 30, o0_30);
    double o0_33 = ((x0_6 * t_M[27]) + (x0_7 * t_M[30]) + (x0_8 * t_M[33]));
    st(0, 33, o0_33);
    double o0_36 = ((x0_0 * t_M[36]) + (x0_1 * t_M[39]) + (x0_2 * t_M[42]));
    st(0, 36, o0_36);
    double o0_39 = ((x0_3 * t_M[36]) + (x0_4 * t_M[39]) + (x0_5 * t_M[42]));
    st(0, 39, o0_39);
    double o0_42 = ((x0_6 * t_M[36]) + (x0_7 * t_M[39]) + (x0_8 * t_M[42]));
    st(0, 42, o0_42);
    double o0_45 = ((x0_0 * t_M[45]) + (x0_1 * t_M[48]) + (x0_2 * t_M[51]));
    st(0, 45, o0_45);
    double o0_48 = ((x0_3 * t_M[45]) + (x0_4 * t_M[48]) + (x0_5 * t_M[51]));
    st(0, 48, o0_48);
    double o0_51 = ((x0_6 * t_M[45]) + (x0_7 * t_M[48]) + (x0_8 * t_M[51]));
    st(0, 51, o0_51);
    __builtin_amdgcn_sched_barrier(0);
    double o0_54 = ((x0_0 * t_M[54]) + (x0_1 * t_M[57]) + (x0_2 * t_M[60]));
    st(0, 54, o0_54);
    double o0_57 = ((x0_3 * t_M[54]) + (x0_4 * t_M[57]) + (x0_5 * t_M[60]));
    st(0, 57, o0_57);
    double o0_60 = ((x0_6 * t_M[54]) + (x0_7 * t_M[57]) + (x0_8 * t_M[60]));
    st(0, 60, o0_60);
    double o0_63 = ((x0_0 * t_M[63]) + (x0_1 * t_M[66]) + (x0_2 * t_M[69]));
    st(0, 63, o0_63);
    double o0_66 = ((x0_3 * t_M[63]) + (x0_4 * t_M[66]) + (x0_5 * t_M[69]));
    st(0, 66, o0_66);
    double o0_69 = ((x0_6 * t_M[63]) + (x0_7 * t_M[66]) + (x0_8 * t_M[69]));
    st(0, 69, o0_69);
    double o0_72 = ((x0_0 * t_M[72]) + (x0_1 * t_M[75]) + (x0_2 * t_M[78]));
    st(0, 72, o0_72);
    double o0_75 = ((x0_3 * t_M[72]) + (x0_4 * t_M[75]) + (x0_5 * t_M[78]));
    st(0, 75, o0_75);
    double o0_78 = ((x0_6 * t_M[72]) + (x0_7 * t_M[75]) + (x0_8 * t_M[78]));
    st(0, 78, o0_78);
    __builtin_amdgcn_sched_barrier(0);
    const double x3_1 = ld(3, 1);
    const double x3_28 = ld(3, 28);
    const double x3_55 = ld(3, 55);
    t_T[1] = ((x2_0 * x3_1) + (x2_1 * x3_28) + (x2_2 * x3_55));
    t_T[28] = ((x2_3 * x3_1) + (x2_4 * x3_28) + (x2_5 * x3_55));
    t_T[55] = ((x2_6 * x3_1) + (x2_7 * x3_28) + (x2_8 * x3_55));
    const double x3_4 = ld(3, 4);
    const double x3_31 = ld(3, 31);
    const double x3_58 = ld(3, 58);
    t_T[4] = ((x2_0 * x3_4) + (x2_1 * x3_31) + (x2_2 * x3_58));
    t_T[31] = ((x2_3 * x3_4) + (x2_4 * x3_31) + (x2_5 * x3_58));
    t_T[58] = ((x2_6 * x3_4) + (x2_7 * x3_31) + (x2_8 * x3_58));
    const double x3_7 = ld(3, 7);
    const double x3_34 = ld(3, 34);
    const double x3_61 = ld(3, 61);
    t_T[7] = ((x2_0 * x3_7) + (x2_1 * x3_34) + (x2_2 * x3_61));
    t_T[34] = ((x2_3 * x3_7) + (x2_4 * x3_34) + (x2_5 * x3_61));
    t_T[61] = ((x2_6 * x3_7) + (x2_7 * x3_34) + (x2_8 * x3_61));
    __builtin_amdgcn_sched_barrier(0);
    const double x3_10 = ld(3, 10);
    const double x3_37 = ld(3, 37);
    const double x3_64 = ld(3, 64);
    t_T[10] = ((x2_0 * x3_10) + (x2_1 * x3_37) + (x2_2 * x3_64));
    t_T[37] = ((x2_3 * x3_10) + (x2_4 * x3_37) + (x2_5 * x3_64));
    t_T[64] = ((x2_6 * x3_10) + (x2_7 * x3_37) + (x2_8 * x3_64));
    const double x3_13 = ld(3, 13);
    const double x3_40 = ld(3, 40);
    const double x3_67 = ld(3, 67);
    t_T[13] = ((x2_0 * x3_13) + (x2_1 * x3_40) + (x2_2 * x3_67));
    t_T[40] = ((x2_3 * x3_13) + (x2_4 * x3_40) + (x2_5 * x3_67));
    t_T[67] = ((x2_6 * x3_13) + (x2_7 * x3_40) + (x2_8 * x3_67));
    const double x3_16 = ld(3, 16);
    const double x3_43 = ld(3, 43);
    const double x3_70 = ld(3, 70);
    t_T[16] = ((x2_0 * x3_16) + (x2_1 * x3_43) + (x2_2 * x3_70));
    t_T[43] = ((x2_3 * x3_16) + (x2_4 * x3_43) + (x2_5 * x3_70));
    t_T[70] = ((x2_6 * x3_16) + (x2_7 * x3_43) + (x2_8 * x3_70));
    __builtin_amdgcn_sched_barrier(0);
    const double x3_19 = ld(3, 19);
    const double x3_46 = ld(3, 46);
    const double x3_73 = ld(3, 73);
    t_T[19] = ((x2_0 * x3_19) + (x2_1 * x3_46) + (x2_2 * x3_73));
    t_T[46] = ((x2_3 * x3_19) + (x2_4 * x3_46) + (x2_5 * x3_73));
    t_T[73] = ((x2_6 * x3_19) + (x2_7 * x3_46) + (x2_8 * x3_73));
    const double x3_22 = ld(3, 22);
    const double x3_49 = ld(3, 49);
    const double x3_76 = ld(3, 76);
    t_T[22] = ((x2_0 * x3_22) + (x2_1 * x3_49) + (x2_2 * x3_76));
    t_T[49] = ((x2_3 * x3_22) + (x2_4 * x3_49) + (x2_5 * x3_76));
    t_T[76] = ((x2_6 * x3_22) + (x2_7 * x3_49) + (x2_8 * x3_76));
    const double x3_25 = ld(3, 25);
    const double x3_52 = ld(3, 52);
    const double x3_79 = ld(3, 79);
    t_T[25] = ((x2_0 * x3_25) + (x2_1 * x3_52) + (x2_2 * x3_79));
    t_T[52] = ((x2_3 * x3_25) + (x2_4 * x3_52) + (x2_5 * x3_79));
    t_T[79] = ((x2_6 * x3_25) + (x2_7 * x3_52) + (x2_8 * x3_79));
    t_M[1] = ((x1_0 * t_T[1]) + (x1_1 * t_T[10]) + (x1_2 * t_T[19]));
    t_M[10] = ((x1_3 * t_T[1]) + (x1_4 * t_T[10]) + (x1_5 * t_T[19]));
    t_M[19] = ((x1_6 * t_T[1]) + (x1_7 * t_T[10]) + (x1_8 * t_T[19]));
    t_M[4] = ((x1_0 * t_T[4]) + (x1_1 * t_T[13]) + (x1_2 * t_T[22]));
    t_M[13] = ((x1_3 * t_T[4]) + (x1_4 * t_T[13]) + (x1_5 * t_T[22]));
    t_M[22] = ((x1_6 * t_T[4]) + (x1_7 * t_T[13]) + (x1_8 * t_T[22]));
    t_M[7] = ((x1_0 * t_T[7]) + (x1_1 * t_T[16]) + (x1_2 * t_T[25]));
    t_M[16] = ((x1_3 * t_T[7]) + (x1_4 * t_T[16]) + (x1_5 * t_T[25]));
    t_M[25] = ((x1_6 * t_T[7]) + (x1_7 * t_T[16]) + (x1_8 * t_T[25]));
    __builtin_amdgcn_sched_barrier(0);
    t_M[28] = ((x1_0 * t_T[28]) + (x1_1 * t_T[37]) + (x1_2 * t_T[46]));
    t_M[37] = ((x1_3 * t_T[28]) + (x1_4 * t_T[37]) + (x1_5 * t_T[46]));
    t_M[46] = ((x1_6 * t_T[28]) + (x1_7 * t_T[37]) + (x1_8 * t_T[46]));
    t_M[31] = ((x1_0 * t_T[31]) + (x1_1 * t_T[40]) + (x1_2 * t_T[49]));
    t_M[40] = ((x1_3 * t_T[31]) + (x1_4 * t_T[40]) + (x1_5 * t_T[49]));
    t_M[49] = ((x1_6 * t_T[31]) + (x1_7 * t_T[40]) + (x1_8 * t_T[49]));
    t_M[34] = ((x1_0 * t_T[34]) + (x1_1 * t_T[43]) + (x1_2 * t_T[52]));
    t_M[43] = ((x1_3 * t_T[34]) + (x1_4 * t_T[43]) + (x1_5 * t_T[52]));
    t_M[52] = ((x1_6 * t_T[34]) + (x1_7 * t_T[43]) + (x1_8 * t_T[52]));
    __builtin_amdgcn_sched_barrier(0);
    t_M[55] = ((x1_0 * t_T[55]) + (x1_1 * t_T[64]) + (x1_2 * t_T[73]));
    t_M[64] = ((x1_3 * t_T[55]) + (x1_4 * t_T[64]) + (x1_5 * t_T[73]));
    t_M[73] = ((x1_6 * t_T[55]) + (x1_7 * t_T[64]) + (x1_8 * t_T[73]));
    t_M[58] = ((x1_0 * t_T[58]) + (x1_1 * t_T[67]) + (x1_2 * t_T[76]));
    t_M[67] = ((x1_3 * t_T[58]) + (x1_4 * t_T[67]) + (x1_5 * t_T[76]));
    t_M[76] = ((x1_6 * t_T[58]) + (x1_7 * t_T[67]) + (x1_8 * t_T[76]));
    t_M[61] = ((x1_0 * t_T[61]) + (x1_1 * t_T[70]) + (x1_2 * t_T[79]));
    t_M[70] = ((x1_3 * t_T[61]) + (x1_4 * t_T[70]) + (x1_5 * t_T[79]));
    t_M[79] = ((x1_6 * t_T[61]) + (x1_7 * t_T[70]) + (x1_8 * t_T[79]));
    double o0_1 = ((x0_0 * t_M[1]) + (x0_1 * t_M[4]) + (x0_2 * t_M[7]));
    st(0, 1, o0_1);
    double o0_4 = ((x0_3 * t_M[1]) + (x0_4 * t_M[4]) + (x0_5 * t_M[7]));
    st(0, 4, o0_4);
    double o0_7 = ((x0_6 * t_M[1]) + (x0_7 * t_M[4]) + (x0_8 * t_M[7]));
    st(0, 7, o0_7);
    double o0_10 = ((x0_0 * t_M[10]) + (x0_1 * t_M[13]) + (x0_2 * t_M[16]));
    st(0, 10, o0_10);
    double o0_13 = ((x0_3 * t_M[10]) + (x0_4 * t_M[13]) + (x0_5 * t_M[16]));
    st(0, 13, o0_13);
    double o0_16 = ((x0_6 * t_M[10]) + (x0_7 * t_M[13]) + (x0_8 * t_M[16]));
    st(0, 16, o0_16);
    double o0_19 = ((x0_0 * t_M[19]) + (x0_1 * t_M[22]) + (x0_2 * t_M[25]));
    st(0, 19, o0_19);
    double o0_22 = ((x0_3 * t_M[19]) + (x0_4 * t_M[22]) + (x0_5 * t_M[25]));
    st(0, 22, o0_22);
    double o0_25 = ((x0_6 * t_M[19]) + (x0_7 * t_M[22]) + (x0_8 * t_M[25]));
    st(0, 25, o0_25);
    __builtin_amdgcn_sched_barrier(0);
    double o0_28 = ((x0_0 * t_M[28]) + (x0_1 * t_M[31]) + (x0_2 * t_M[34]));
    st(0, 28, o0_28);
    double o0_31 = ((x0_3 * t_M[28]) + (x0_4 * t_M[31]) + (x0_5 * t_M[34]));
    st(0, 31, o0_31);
    double o0_34 = ((x0_6 * t_M[28]) + (x0_7 * t_M[31]) + (x0_8 * t_M[34]));
    st(0, 34, o0_34);
    double o0_37 = ((x0_0 * t_M[37]) + (x0_1 * t_M[40]) + (x0_2 * t_M[43]));
    st(0, 37, o0_37);
    double o0_40 = ((x0_3 * t_M[37]) + (x0_4 * t_M[40]) + (x0_5 * t_M[43]));
    st(0, 40, o0_40);
    double o0_43 = ((x0_6 * t_M[37]) + (x0_7 * t_M[40]) + (x0_8 * t_M[43]));
    st(0, 43, o0_43);
    double o0_46 = ((x0_0 * t_M[46]) + (x0_1 * t_M[49]) + (x0_2 * t_M[52]));
    st(0, 46, o0_46);
    double o0_49 = ((x0_3 * t_M[46]) + (x0_4 * t_M[49]) + (x0_5 * t_M[52]));
    st(0, 49, o0_49);
    double o0_52 = ((x0_6 * t_M[46]) + (x0_7 * t_M[49]) + (x0_8 * t_M[52]));
    st(0, 52, o0_52);
    __builtin_amdgcn_sched_barrier(0);
    double o0_55 = ((x0_0 * t_M[55]) + (x0_1 * t_M[58]) + (x0_2 * t_M[61]));
    st(0, 55, o0_55);
    double o0_58 = ((x0_3 * t_M[55]) + (x0_4 * t_M[58]) + (x0_5 * t_M[61]));
    st(0, 58, o0_58);
    double o0_61 = ((x0_6 * t_M[55]) + (x0_7 * t_M[58]) + (x0_8 * t_M[61]));
    st(0, 61, o0_61);
    double o0_64 = ((x0_0 * t_M[64]) + (x0_1 * t_M[67]) + (x0_2 * t_M[70]));
    st(0, 64, o0_64);
    double o0_67 = ((x0_3 * t_M[64]) + (x0_4 * t_M[67]) + (x0_5 * t_M[70]));
    st(0, 67, o0_67);
    double o0_70 = ((x0_6 * t_M[64]) + (x0_7 * t_M[67]) + (x0_8 * t_M[70]));
    st(0, 70, o0_70);
    double o0_73 = ((x0_0 * t_M[73]) + (x0_1 * t_M[76]) + (x0_2 * t_M[79]));
    st(0, 73, o0_73);
    double o0_76 = ((x0_3 * t_M[73]) + (x0_4 * t_M[76]) + (x0_5 * t_M[79]));
    st(0, 76, o0_76);
    double o0_79 = ((x0_6 * t_M[73]) + (x0_7 * t_M[76]) + (x0_8 * t_M[79]));
    st(0, 79, o0_79);
    __builtin_amdgcn_sched_barrier(0);
    const double x3_2 = ld(3, 2);
    const double x3_29 = ld(3, 29);
    const double x3_56 = ld(3, 56);
    t_T[2] = ((x2_0 * x3_2) + (x2_1 * x3_29) + (x2_2 * x3_56));
    t_T[29] = ((x2_3 * x3_2) + (x2_4 * x3_29) + (x2_5 * x3_56));
    t_T[56] = ((x2_6 * x3_2) + (x2_7 * x3_29) + (x2_8 * x3_56));
    const double x3_5 = ld(3, 5);
    const double x3_32 = ld(3, 32);
    const double x3_59 = ld(3, 59);
    t_T[5] = ((x2_0 * x3_5) + (x2_1 * x3_32) + (x2_2 * x3_59));
    t_T[32] = ((x2_3 * x3_5) + (x2_4 * x3_32) + (x2_5 * x3_59));
    t_T[59] = ((x2_6 * x3_5) + (x2_7 * x3_32) + (x2_8 * x3_59));
    const double x3_8 = ld(3, 8);
    const double x3_35 = ld(3, 35);
    const double x3_62 = ld(3, 62);
    t_T[8] = ((x2_0 * x3_8) + (x2_1 * x3_35) + (x2_2 * x3_62));
    t_T[35] = ((x2_3 * x3_8) + (x2_4 * x3_35) + (x2_5 * x3_62));
    t_T[62] = ((x2_6 * x3_8) + (x2_7 * x3_35) + (x2_8 * x3_62));
    __builtin_amdgcn_sched_barrier(0);
    const double x3_11 = ld(3, 11);
    const double x3_38 = ld(3, 38);
    const double x3_65 = ld(3, 65);
    t_T[11] = ((x2_0 * x3_11) + (x2_1 * x3_38) + (x2_2 * x3_65));
    t_T[38] = ((x2_3 * x3_11) + (x2_4 * x3_38) + (x2_5 * x3_65));
    t_T[65] = ((x2_6 * x3_11) + (x2_7 * x3_38) + (x2_8 * x3_65));
    const double x3_14 = ld(3, 14);
    const double x3_41 = ld(3, 41);
    const double x3_68 = ld(3, 68);
    t_T[14] = ((x2_0 * x3_14) + (x2_1 * x3_41) + (x2_2 * x3_68));
    t_T[41] = ((x2_3 * x3_14) + (x2_4 * x3_41) + (x2_5 * x3_68));
    t_T[68] = ((x2_6 * x3_14) + (x2_7 * x3_41) + (x2_8 * x3_68));
    const double x3_17 = ld(3, 17);
    const double x3_44 = ld(3, 44);
    const double x3_71 = ld(3, 71);
    t_T[17] = ((x2_0 * x3_17) + (x2_1 * x3_44) + (x2_2 * x3_71));
    t_T[44] = ((x2_3 * x3_17) + (x2_4 * x3_44) + (x2_5 * x3_71));
    t_T[71] = ((x2_6 * x3_17) + (x2_7 * x3_44) + (x2_8 * x3_71));
    __builtin_amdgcn_sched_barrier(0);
    const double x3_20 = ld(3, 20);
    const double x3_47 = ld(3, 47);
    const double x3_74 = ld(3, 74);
    t_T[20] = ((x2_0 * x3_20) + (x2_1 * x3_47) + (x2_2 * x3_74));
    t_T[47] = ((x2_3 * x3_20) + (x2_4 * x3_47) + (x2_5 * x3_74));
    t_T[74] = ((x2_6 * x3_20) + (x2_7 * x3_47) + (x2_8 * x3_74));
    const double x3_23 = ld(3, 23);
    const double x3_50 = ld(3, 50);
    const double x3_77 = ld(3, 77);
    t_T[23] = ((x2_0 * x3_23) + (x2_1 * x3_50) + (x2_2 * x3_77));
    t_T[50] = ((x2_3 * x3_23) + (x2_4 * x3_50) + (x2_5 * x3_77));
    t_T[77] = ((x2_6 * x3_23) + (x2_7 * x3_50) + (x2_8 * x3_77));
    const double x3_26 = ld(3, 26);
    const double x3_53 = ld(3, 53);
    const double x3_80 = ld(3, 80);
    t_T[26] = ((x2_0 * x3_26) + (x2_1 * x3_53) + (x2_2 * x3_80));
    t_T[53] = ((x2_3 * x3_26) + (x2_4 * x3_53) + (x2_5 * x3_80));
    t_T[80] = ((x2_6 * x3_26) + (x2_7 * x3_53) + (x2_8 * x3_80));
    t_M[2] = ((x1_0 * t_T[2]) + (x1_1 * t_T[11]) + (x1_2 * t_T[20]));
    t_M[11] = ((x1_3 * t_T[2]) + (x1_4 * t_T[11]) + (x1_5 * t_T[20]));
    t_M[20] = ((x1_6 * t_T[2]) + (x1_7 * t_T[11]) + (x1_8 * t_T[20]));
    t_M[5] = ((x1_0 * t_T[5]) + (x1_1 * t_T[14]) + (x1_2 * t_T[23]));
    t_M[14] = ((x1_3 * t_T[5]) + (x1_4 * t_T[14]) + (x1_5 * t_T[23]));
    t_M[23] = ((x1_6 * t_T[5]) + (x1_7 * t_T[14]) + (x1_8 * t_T[23]));
    t_M[8] = ((x1_0 * t_T[8]) + (x1_1 * t_T[17]) + (x1_2 * t_T[26]));
    t_M[17] = ((x1_3 * t_T[8]) + (x1_4 * t_T[17]) + (x1_5 * t_T[26]));
    t_M[26] = ((x1_6 * t_T[8]) + (x1_7 * t_T[17]) + (x1_8 * t_T[26]));
    __builtin_amdgcn_sched_barrier(0);
    t_M[29] = ((x1_0 * t_T[29]) + (x1_1 * t_T[38]) + (x1_2 * t_T[47]));
    t_M[38] = ((x1_3 * t_T[29]) + (x1_4 * t_T[38]) + (x1_5 * t_T[47]));
    t_M[47] = ((x1_6 * t_T[29]) + (x1_7 * t_T[38]) + (x1_8 * t_T[47]));
    t_M[32] = ((x1_0 * t_T[32]) + (x1_1 * t_T[41]) + (x1_2 * t_T[50]));
    t_M[41] = ((x1_3 * t_T[32]) + (x1_4 * t_T[41]) + (x1_5 * t_T[50]));
    t_M[50] = ((x1_6 * t_T[32]) + (x1_7 * t_T[41]) + (x1_8 * t_T[50]));
    t_M[35] = ((x1_0 * t_T[35]) + (x1_1 * t_T[44]) + (x1_2 * t_T[53]));
    t_M[44] = ((x1_3 * t_T[35]) + (x1_4 * t_T[44]) + (x1_5 * t_T[53]));
    t_M[53] = ((x1_6 * t_T[35]) + (x1_7 * t_T[44]) + (x1_8 * t_T[53]));
    __builtin_amdgcn_sched_barrier(0);
    t_M[56] = ((x1_0 * t_T[56]) + (x1_1 * t_T[65]) + (x1_2 * t_T[74]));
    t_M[65] = ((x1_3 * t_T[56]) + (x1_4 * t_T[65]) + (x1_5 * t_T[74]));
    t_M[74] = ((x1_6 * t_T[56]) + (x1_7 * t_T[65]) + (x1_8 * t_T[74]));
    t_M[59] = ((x1_0 * t_T[59]) + (x1_1 * t_T[68]) + (x1_2 * t_T[77]));
    t_M[68] = ((x1_3 * t_T[59]) + (x1_4 * t_T[68]) + (x1_5 * t_T[77]));
    t_M[77] = ((x1_6 * t_T[59]) + (x1_7 * t_T[68]) + (x1_8 * t_T[77]));
    t_M[62] = ((x1_0 * t_T[62]) + (x1_1 * t_T[71]) + (x1_2 * t_T[80]));
    t_M[71] = ((x1_3 * t_T[62]) + (x1_4 * t_T[71]) + (x1_5 * t_T[80]));
    t_M[80] = ((x1_6 * t_T[62]) + (x1_7 * t_T[71]) + (x1_8 * t_T[80]));
    double o0_2 = ((x0_0 * t_M[2]) + (x0_1 * t_M[5]) + (x0_2 * t_M[8]));
    st(0, 2, o0_2);
    double o0_5 = ((x0_3 * t_M[2]) + (x0_4 * t_M[5]) + (x0_5 * t_M[8]));
    st(0, 5, o0_5);
    double o0_8 = ((x0_6 * t_M[2]) + (x0_7 * t_M[5]) + (x0_8 * t_M[8]));
    st(0, 8, o0_8);
    double o0_11 = ((x0_0 * t_M[11]) + (x0_1 * t_M[14]) + (x0_2 * t_M[17]));
    st(0, 11, o0_11);
    double o0_14 = ((x0_3 * t_M[11]) + (x0_4 * t_M[14]) + (x0_5 * t_M[17]));
    st(0, 14, o0_14);
    double o0_17 = ((x0_6 * t_M[11]) + (x0_7 * t_M[14]) + (x0_8 * t_M[17]));
    st(0, 17, o0_17);
    double o0_20 = ((x0_0 * t_M[20]) + (x0_1 * t_M[23]) + (x0_2 * t_M[26]));
    st(0, 20, o0_20);
    double o0_23 = ((x0_3 * t_M[20]) + (x0_4 * t_M[23]) + (x0_5 * t_M[26]));
    st(0, 23, o0_23);
    double o0_26 = ((x0_6 * t_M[20]) + (x0_7 * t_M[23]) + (x0_8 * t_M[26]));
    st(0, 26, o0_26);
    __builtin_amdgcn_sched_barrier(0);
    double o0_29 = ((x0_0 * t_M[29]) + (x0_1 * t_M[32]) + (x0_2 * t_M[35]));
    st(0, 29, o0_29);
    double o0_32 = ((x0_3 * t_M[29]) + (x0_4 * t_M[32]) + (x0_5 * t_M[35]));
    st(0, 32, o0_32);
    double o0_35 = ((x0_6 * t_M[29]) + (x0_7 * t_M[32]) + (x0_8 * t_M[35]));
    st(0, 35, o0_35);
    double o0_38 = ((x0_0 * t_M[38]) + (x0_1 * t_M[41]) + (x0_2 * t_M[44]));
    st(0, 38, o0_38);
    double o0_41 = ((x0_3 * t_M[38]) + (x0_4 * t_M[41]) + (x0_5 * t_M[44]));
    st(0, 41, o0_41);
    double o0_44 = ((x0_6 * t_M[38]) + (x0_7 * t_M[41]) + (x0_8 * t_M[44]));
    st(0, 44, o0_44);
    double o0_47 = ((x0_0 * t_M[47]) + (x0_1 * t_M[50]) + (x0_2 * t_M[53]));
    st(0, 47, o0_47);
    double o0_50 = ((x0_3 * t_M[47]) + (x0_4 * t_M[50]) + (x0_5 * t_M[53]));
    st(0, 50, o0_50);
    double o0_53 = ((x0_6 * t_M[47]) + (x0_7 * t_M[50]) + (x0_8 * t_M[53]));
    st(0, 53, o0_53);
    __builtin_amdgcn_sched_barrier(0);
    double o0_56 = ((x0_0 * t_M[56]) + (x0_1 * t_M[59]) + (x0_2 * t_M[62]));
    st(0, 56, o0_56);
    double o0_59 = ((x0_3 * t_M[56]) + (x0_4 * t_M[59]) + (x0_5 * t_M[62]));
    st(0, 59, o0_59);
    double o0_62 = ((x0_6 * t_M[56]) + (x0_7 * t_M[59]) + (x0_8 * t_M[62]));
    st(0, 62, o0_62);
    double o0_65 = ((x0_0 * t_M[65]) + (x0_1 * t_M[68]) + (x0_2 * t_M[71]));
    st(0, 65, o0_65);
    double o0_68 = ((x0_3 * t_M[65]) + (x0_4 * t_M[68]) + (x0_5 * t_M[71]));
    st(0, 68, o0_68);
    double o0_71 = ((x0_6 * t_M[65]) + (x0_7 * t_M[68]) + (x0_8 * t_M[71]));
    st(0, 71, o0_71);
    double o0_74 = ((x0_0 * t_M[74]) + (x0_1 * t_M[77]) + (x0_2 * t_M[80]));
    st(0, 74, o0_74);
    double o0_77 = ((x0_3 * t_M[74]) + (x0_4 * t_M[77]) + (x0_5 * t_M[80]));
    st(0, 77, o0_77);
    double o0_80 = ((x0_6 * t_M[74]) + (x0_7 * t_M[77]) + (x0_8 * t_M[80]));
    st(0, 80, o0_80);
  }
};

// lst_sym_contract: C_(ab) = sum_c A_ac B_cb, symmetric left-hand side (Sec. 4, rank 2 contraction example)
struct Gen_lst_sym_contract {
  static constexpr bool kStream = true;
  static constexpr int NF_IN = 2, NF_OUT = 1;
  static constexpr int fin[NF_IN] = {16, 16};
  static constexpr int fout[NF_OUT] = {10};
  static constexpr int NIN = 32, NOUT = 10;
  template <class L, class S>
  __device__ static inline void stream(L&& ld, S&& st) {
    const double x0_0 = ld(0, 0);
    const double x0_1 = ld(0, 1);
    const double x0_2 = ld(0, 2);
    const double x0_3 = ld(0, 3);
    const double x0_4 = ld(0, 4);
    const double x0_5 = ld(0, 5);
    const double x0_6 = ld(0, 6);
    const double x0_7 = ld(0, 7);
    const double x0_8 = ld(0, 8);
    const double x0_9 = ld(0, 9);
    const double x0_10 = ld(0, 10);
    const double x0_11 = ld(0, 11);
    const double x0_12 = ld(0, 12);
    const double x0_13 = ld(0, 13);
    const double x0_14 = ld(0, 14);
    const double x0_15 = ld(0, 15);
    const double x1_0 = ld(1, 0);
    const double x1_1 = ld(1, 1);
    const double x1_2 = ld(1, 2);
    const double x1_3 = ld(1, 3);
    const double x1_4 = ld(1, 4);
    const double x1_5 = ld(1, 5);
    const double x1_6 = ld(1, 6);
    const double x1_7 = ld(1, 7);
    const double x1_8 = ld(1, 8);
    const double x1_9 = ld(1, 9);
    const double x1_10 = ld(1, 10);
    const double x1_11 = ld(1, 11);
    const double x1_12 = ld(1, 12);
    const double x1_13 = ld(1, 13);
    const double x1_14 = ld(1, 14);
    const double x1_15 = ld(1, 15);
    // C(a,b) = Sum(c, (A(a,c) * B(c,b)))
    double o0_0 = ((x0_0 * x1_0) + (x0_1 * x1_4) + (x0_2 * x1_8) + (x0_3 * x1_12));
    st(0, 0, o0_0);
    double o0_1 = ((x0_4 * x1_0) + (x0_5 * x1_4) + (x0_6 * x1_8) + (x0_7 * x1_12));
    st(0, 1, o0_1);
    double o0_4 = ((x0_4 * x1_1) + (x0_5 * x1_5) + (x0_6 * x1_9) + (x0_7 * x1_13));
    st(0, 4, o0_4);
    double o0_2 = ((x0_8 * x1_0) + (x0_9 * x1_4) + (x0_10 * x1_8) + (x0_11 * x1_12));
    st(0, 2, o0_2);
    double o0_5 = ((x0_8 * x1_1) + (x0_9 * x1_5) + (x0_10 * x1_9) + (x0_11 * x1_13));
    st(0, 5, o0_5);
    double o0_7 = ((x0_8 * x1_2) + (x0_9 * x1_6) + (x0_10 * x1_10) + (x0_11 * x1_14));
    st(0, 7, o0_7);
    double o0_3 = ((x0_12 * x1_0) + (x0_13 * x1_4) + (x0_14 * x1_8) + (x0_15 * x1_12));
    st(0, 3, o0_3);
    double o0_6 = ((x0_12 * x1_1) + (x0_13 * x1_5) + (x0_14 * x1_9) + (x0_15 * x1_13));
    st(0, 6, o0_6);
    double o0_8 = ((x0_12 * x1_2) + (x0_13 * x1_6) + (x0_14 * x1_10) + (x0_15 * x1_14));
    st(0, 8, o0_8);
    double o0_9 = ((x0_12 * x1_3) + (x0_13 * x1_7) + (x0_14 * x1_11) + (x0_15 * x1_15));
    st(0, 9, o0_9);
  }
};

// lst_fixed_offset: D_(i0) = sum_c E_(i+1)c F_c0, fixed and offset indices (Sec. 4, second contraction example)
struct Gen_lst_fixed_offset {
  static constexpr bool kStream = true;
  static constexpr int NF_IN = 2, NF_OUT = 1;
  static constexpr int fin[NF_IN] = {16, 16};
  static constexpr int fout[NF_OUT] = {10};
  static constexpr int NIN = 32, NOUT = 10;
  template <class L, class S>
  __device__ static inline void stream(L&& ld, S&& st) {
    const double x0_4 = ld(0, 4);
    const double x0_5 = ld(0, 5);
    const double x0_6 = ld(0, 6);
    const double x0_7 = ld(0, 7);
    const double x0_8 = ld(0, 8);
    const double x0_9 = ld(0, 9);
    const double x0_10 = ld(0, 10);
    const double x0_11 = ld(0, 11);
    const double x0_12 = ld(0, 12);
    const double x0_13 = ld(0, 13);
    const double x0_14 = ld(0, 14);
    const double x0_15 = ld(0, 15);
    const double x1_0 = ld(1, 0);
    const double x1_4 = ld(1, 4);
    const double x1_8 = ld(1, 8);
    const double x1_12 = ld(1, 12);
    // D(i,0) = Sum(c, (E(i+1,c) * F(c,0)))
    double o0_0 = ((x0_4 * x1_0) + (x0_5 * x1_4) + (x0_6 * x1_8) + (x0_7 * x1_12));
    st(0, 0, o0_0);
    double o0_1 = ((x0_8 * x1_0) + (x0_9 * x1_4) + (x0_10 * x1_8) + (x0_11 * x1_12));
    st(0, 1, o0_1);
    double o0_2 = ((x0_12 * x1_0) + (x0_13 * x1_4) + (x0_14 * x1_8) + (x0_15 * x1_12));
    st(0, 2, o0_2);
  }
};

// spacetime_split: spatial metric and shift from the spacetime metric psi_ab (Sec. 2.2)
struct Gen_spacetime_split {
  static constexpr bool kStream = true;
  static constexpr int NF_IN = 1, NF_OUT = 2;
  static constexpr int fin[NF_IN] = {10};
  static constexpr int fout[NF_OUT] = {6, 3};
  static constexpr int NIN = 10, NOUT = 9;
  template <class L, class S>
  __device__ static inline void stream(L&& ld, S&& st) {
    const double x0_1 = ld(0, 1);
    const double x0_2 = ld(0, 2);
    const double x0_3 = ld(0, 3);
    const double x0_4 = ld(0, 4);
    const double x0_5 = ld(0, 5);
    const double x0_6 = ld(0, 6);
    const double x0_7 = ld(0, 7);
    const double x0_8 = ld(0, 8);
    const double x0_9 = ld(0, 9);
    // g(i,j) = psi(i+1,j+1)
    double o0_0 = x0_4;
    st(0, 0, o0_0);
    double o0_1 = x0_5;
    st(0, 1, o0_1);
    double o0_3 = x0_7;
    st(0, 3, o0_3);
    double o0_2 = x0_6;
    st(0, 2, o0_2);
    double o0_4 = x0_8;
    st(0, 4, o0_4);
    double o0_5 = x0_9;
    st(0, 5, o0_5);
    // beta(i) = psi(i+1,0)
    double o1_0 = x0_1;
    st(1, 0, o1_0);
    double o1_1 = x0_2;
    st(1, 1, o1_1);
    double o1_2 = x0_3;
    st(1, 2, o1_2);
  }
};

}  // namespace tl

extern "C" {

tl_status tlg_christoffel(int64_t n, const tl_cfield* in, int32_t nin, const tl_field* out, int32_t nout, void* stream, const tl_tune* tune) {
  static const int32_t kIn[] = {6, 18};
  static const int32_t kOut[] = {18};
  return tl::run_generated("christoffel", n, in, nin, kIn, 2, out, nout, kOut,
                           1, stream, tune, &tl::launch_op<tl::Gen_christoffel>);
}

tl_status tlg_cov_deriv(int64_t n, const tl_cfield* in, int32_t nin, const tl_field* out, int32_t nout, void* stream, const tl_tune* tune) {
  static const int32_t kIn[] = {9, 18, 3};
  static const int32_t kOut[] = {9};
  return tl::run_generated("cov_deriv", n, in, nin, kIn, 3, out, nout, kOut,
                           1, stream, tune, &tl::launch_op<tl::Gen_cov_deriv>);
}

tl_status tlg_dtg(int64_t n, const tl_cfield* in, int32_t nin, const tl_field* out, int32_t nout, void* stream, const tl_tune* tune) {
  static const int32_t kIn[] = {1, 6, 9};
  static const int32_t kOut[] = {6};
  return tl::run_generated("dtg", n, in, nin, kIn, 3, out, nout, kOut,
                           1, stream, tune, &tl::launch_op<tl::Gen_dtg>);
}

tl_status tlg_dtg_chain_invg(int64_t n, const tl_cfield* in, int32_t nin, const tl_field* out, int32_t nout, void* stream, const tl_tune* tune) {
  static const int32_t kIn[] = {6, 18, 9, 3, 1, 6};
  static const int32_t kOut[] = {6};
  return tl::run_generated("dtg_chain_invg", n, in, nin, kIn, 6, out, nout, kOut,
                           1, stream, tune, &tl::launch_op<tl::Gen_dtg_chain_invg>);
}

tl_status tlg_kij(int64_t n, const tl_cfield* in, int32_t nin, const tl_field* out, int32_t nout, void* stream, const tl_tune* tune) {
  static const int32_t kIn[] = {1, 6, 3};
  static const int32_t kOut[] = {6};
  return tl::run_generated("kij", n, in, nin, kIn, 3, out, nout, kOut,
                           1, stream, tune, &tl::launch_op<tl::Gen_kij>);
}

tl_status tlg_assign1(int64_t n, const tl_cfield* in, int32_t nin, const tl_field* out, int32_t nout, void* stream, const tl_tune* tune) {
  static const int32_t kIn[] = {3};
  static const int32_t kOut[] = {3};
  return tl::run_generated("assign1", n, in, nin, kIn, 1, out, nout, kOut,
                           1, stream, tune, &tl::launch_op<tl::Gen_assign1>);
}

tl_status tlg_assign2(int64_t n, const tl_cfield* in, int32_t nin, const tl_field* out, int32_t nout, void* stream, const tl_tune* tune) {
  static const int32_t kIn[] = {9};
  static const int32_t kOut[] = {9};
  return tl::run_generated("assign2", n, in, nin, kIn, 1, out, nout, kOut,
                           1, stream, tune, &tl::launch_op<tl::Gen_assign2>);
}

tl_status tlg_assign3(int64_t n, const tl_cfield* in, int32_t nin, const tl_field* out, int32_t nout, void* stream, const tl_tune* tune) {
  static const int32_t kIn[] = {27};
  static const int32_t kOut[] = {27};
  return tl::run_generated("assign3", n, in, nin, kIn, 1, out, nout, kOut,
                           1, stream, tune, &tl::launch_op<tl::Gen_assign3>);
}

tl_status tlg_add1(int64_t n, const tl_cfield* in, int32_t nin, const tl_field* out, int32_t nout, void* stream, const tl_tune* tune) {
  static const int32_t kIn[] = {3, 3};
  static const int32_t kOut[] = {3};
  return tl::run_generated("add1", n, in, nin, kIn, 2, out, nout, kOut,
                           1, stream, tune, &tl::launch_op<tl::Gen_add1>);
}

tl_status tlg_add2(int64_t n, const tl_cfield* in, int32_t nin, const tl_field* out, int32_t nout, void* stream, const tl_tune* tune) {
  static const int32_t kIn[] = {3, 3, 3};
  static const int32_t kOut[] = {3};
  return tl::run_generated("add2", n, in, nin, kIn, 3, out, nout, kOut,
                           1, stream, tune, &tl::launch_op<tl::Gen_add2>);
}

tl_status tlg_add3(int64_t n, const tl_cfield* in, int32_t nin, const tl_field* out, int32_t nout, void* stream, const tl_tune* tune) {
  static const int32_t kIn[] = {3, 3, 3, 3};
  static const int32_t kOut[] = {3};
  return tl::run_generated("add3", n, in, nin, kIn, 4, out, nout, kOut,
                           1, stream, tune, &tl::launch_op<tl::Gen_add3>);
}

tl_status tlg_mult1(int64_t n, const tl_cfield* in, int32_t nin, const tl_field* out, int32_t nout, void* stream, const tl_tune* tune) {
  static const int32_t kIn[] = {3, 3};
  static const int32_t kOut[] = {9};
  return tl::run_generated("mult1", n, in, nin, kIn, 2, out, nout, kOut,
                           1, stream, tune, &tl::launch_op<tl::Gen_mult1>);
}

tl_status tlg_mult2(int64_t n, const tl_cfield* in, int32_t nin, const tl_field* out, int32_t nout, void* stream, const tl_tune* tune) {
  static const int32_t kIn[] = {3, 3, 3};
  static const int32_t kOut[] = {27};
  return tl::run_generated("mult2", n, in, nin, kIn, 3, out, nout, kOut,
                           1, stream, tune, &tl::launch_op<tl::Gen_mult2>);
}

tl_status tlg_mult3(int64_t n, const tl_cfield* in, int32_t nin, const tl_field* out, int32_t nout, void* stream, const tl_tune* tune) {
  static const int32_t kIn[] = {3, 3, 3, 3};
  static const int32_t kOut[] = {81};
  return tl::run_generated("mult3", n, in, nin, kIn, 4, out, nout, kOut,
                           1, stream, tune, &tl::launch_op<tl::Gen_mult3>);
}

tl_status tlg_contract1(int64_t n, const tl_cfield* in, int32_t nin, const tl_field* out, int32_t nout, void* stream, const tl_tune* tune) {
  static const int32_t kIn[] = {9, 81};
  static const int32_t kOut[] = {81};
  return tl::run_generated("contract1", n, in, nin, kIn, 2, out, nout, kOut,
                           1, stream, tune, &tl::launch_op<tl::Gen_contract1>);
}

tl_status tlg_contract2(int64_t n, const tl_cfield* in, int32_t nin, const tl_field* out, int32_t nout, void* stream, const tl_tune* tune) {
  static const int32_t kIn[] = {9, 9, 81};
  static const int32_t kOut[] = {81};
  return tl::run_generated("contract2", n, in, nin, kIn, 3, out, nout, kOut,
                           1, stream, tune, &tl::launch_op<tl::Gen_contract2>);
}

tl_status tlg_contract3(int64_t n, const tl_cfield* in, int32_t nin, const tl_field* out, int32_t nout, void* stream, const tl_tune* tune) {
  static const int32_t kIn[] = {9, 9, 9, 81};
  static const int32_t kOut[] = {81};
  return tl::run_generated("contract3", n, in, nin, kIn, 4, out, nout, kOut,
                           1, stream, tune, &tl::launch_op<tl::Gen_contract3>);
}

tl_status tlg_lst_sym_contract(int64_t n, const tl_cfield* in, int32_t nin, const tl_field* out, int32_t nout, void* stream, const tl_tune* tune) {
  static const int32_t kIn[] = {16, 16};
  static const int32_t kOut[] = {10};
  return tl::run_generated("lst_sym_contract", n, in, nin, kIn, 2, out, nout, kOut,
                           1, stream, tune, &tl::launch_op<tl::Gen_lst_sym_contract>);
}

tl_status tlg_lst_fixed_offset(int64_t n, const tl_cfield* in, int32_t nin, const tl_field* out, int32_t nout, void* stream, const tl_tune* tune) {
  static const int32_t kIn[] = {16, 16};
  static const int32_t kOut[] = {10};
  return tl::run_generated("lst_fixed_offset", n, in, nin, kIn, 2, out, nout, kOut,
                           1, stream, tune, &tl::launch_op<tl::Gen_lst_fixed_offset>);
}

tl_status tlg_spacetime_split(int64_t n, const tl_cfield* in, int32_t nin, const tl_field* out, int32_t nout, void* stream, const tl_tune* tune) {
  static const int32_t kIn[] = {10};
  static const int32_t kOut[] = {6, 3};
  return tl::run_generated("spacetime_split", n, in, nin, kIn, 1, out, nout, kOut,
                           2, stream, tune, &tl::launch_op<tl::Gen_spacetime_split>);
}

}  // extern "C"
