"""The expressions compiled into the library by the code generator.

Each is written the way the paper writes its TLoops expressions, with the
citation of the passage it comes from.  The build regenerates
csrc/generated/tlg_kernels.hip, include/tl_generated.h and generated.json from
this list (``python -m paper_1804_10120_amd.codegen``).
"""
from __future__ import annotations

from .dsl import Program, Sum, Tensor, indices


def programs():
    i, j, k, l, m = indices("i j k l m")
    a, b, c = indices("a b c", 4)

    # spatial tensors, layouts as in tl.h
    g = Tensor("g", (3, 3), sym=[(0, 1)])
    Invg = Tensor("Invg", (3, 3), sym=[(0, 1)])
    dg = Tensor("dg", (3, 3, 3), sym=[(1, 2)])          # dg(k,i,j) = d_k g_ij
    Gamma = Tensor("Gamma", (3, 3, 3), sym=[(1, 2)])    # Gamma(i,j,k) = Gamma^i_jk
    beta = Tensor("beta", (3,))
    dbeta = Tensor("dbeta", (3, 3))                     # dbeta(j,i) = d_j beta_i
    nabla = Tensor("nabla", (3, 3))                     # nabla(j,i) = nabla_j beta_i
    K = Tensor("K", (3, 3), sym=[(0, 1)])
    alpha = Tensor("alpha", ())
    dtg = Tensor("dtg", (3, 3), sym=[(0, 1)])

    christoffel = (0.5 * Sum(l, Invg[i, l] * (dg[k, j, l] + dg[j, l, k] - dg[l, j, k])))
    out = []

    out.append(Program("christoffel", "Christoffel symbols from g^ij and d_k g_ij "
                                      "(Sec. 1, eq:SpatialChristoffel)")
               .let(Gamma[i, j, k], christoffel))
    out.append(Program("cov_deriv", "covariant derivative of the shift (Sec. 1, footnote)")
               .let(nabla[j, i], dbeta[j, i] - Sum(k, Gamma[k, i, j] * beta[k])))
    out.append(Program("dtg", "metric evolution from nabla beta (Sec. 1, eq:dtg_ij)")
               .let(dtg[i, j], -2.0 * alpha[()] * K[i, j] + nabla[i, j] + nabla[j, i]))
    out.append(Program("dtg_chain_invg",
                       "Christoffel symbols, covariant derivative and metric evolution in one "
                       "kernel, Gamma and nabla beta in registers (Sec. 1)")
               .temp(Gamma, nabla)
               .let(Gamma[i, j, k], christoffel)
               .let(nabla[j, i], dbeta[j, i] - Sum(k, Gamma[k, i, j] * beta[k]))
               .let(dtg[i, j], -2.0 * alpha[()] * K[i, j] + nabla[i, j] + nabla[j, i]))

    Kout = Tensor("K", (3, 3), sym=[(0, 1)])
    out.append(Program("kij", "K_ij = 2 alpha g_ij + beta_i beta_j (Sec. 5.1, eq:Kij)")
               .let(Kout[i, j], 2.0 * alpha[()] * g[i, j] + beta[i] * beta[j]))

    # the rest of the Sec. 5.1 benchmark family, inputs in the order written
    n_, o_ = indices("n o")
    B1, C1, D1, E1 = (Tensor(x, (3,)) for x in "BCDE")
    A1 = Tensor("A", (3,))
    A2 = Tensor("A", (3, 3))
    A3 = Tensor("A", (3, 3, 3))
    B2, B3 = Tensor("B", (3, 3)), Tensor("B", (3, 3, 3))
    out.append(Program("assign1", "A_i = B_i (Sec. 5.1, eq:Assign1)").let(A1[i], B1[i]))
    out.append(Program("assign2", "A_ij = B_ij (Sec. 5.1, eq:Assign2)").let(A2[i, j], B2[i, j]))
    out.append(Program("assign3", "A_ijk = B_ijk (Sec. 5.1, eq:Assign3)")
               .let(A3[i, j, k], B3[i, j, k]))
    out.append(Program("add1", "A_i = B_i + C_i (Sec. 5.1, eq:Add1)")
               .let(A1[i], B1[i] + C1[i]))
    out.append(Program("add2", "A_i = B_i + C_i + D_i (Sec. 5.1, eq:Add2)")
               .let(A1[i], B1[i] + C1[i] + D1[i]))
    out.append(Program("add3", "A_i = B_i + C_i + D_i + E_i (Sec. 5.1, eq:Add3)")
               .let(A1[i], B1[i] + C1[i] + D1[i] + E1[i]))
    out.append(Program("mult1", "A_ij = B_i C_j (Sec. 5.1, eq:Mult1)")
               .let(A2[i, j], B1[i] * C1[j]))
    out.append(Program("mult2", "A_ijk = B_i C_j D_k (Sec. 5.1, eq:Mult2)")
               .let(A3[i, j, k], B1[i] * C1[j] * D1[k]))
    A4 = Tensor("A", (3, 3, 3, 3))
    out.append(Program("mult3", "A_ijkl = B_i C_j D_k E_l (Sec. 5.1, eq:Mult3)")
               .let(A4[i, j, k, l], B1[i] * C1[j] * D1[k] * E1[l]))

    B = Tensor("B", (3, 3))
    C = Tensor("C", (3, 3))
    Dm = Tensor("D", (3, 3))
    E = Tensor("E", (3, 3, 3, 3))
    out.append(Program("contract1", "A_ijkl = B_i^m E_mjkl (Sec. 5.1, eq:Contract1)")
               .let(A4[i, j, k, l], Sum(m, B[i, m] * E[m, j, k, l])))
    out.append(Program("contract2", "A_ijkl = C_j^n B_i^m E_mnkl (Sec. 5.1, eq:Contract2)")
               .let(A4[i, j, k, l], Sum(m, Sum(n_, C[j, n_] * B[i, m] * E[m, n_, k, l]))))
    # the triple contraction one index at a time, slice by slice in l: for each
    # l, T_ino = B_i^m E_mnol, then M_ijo = C_j^n T_ino, then A_ijkl = D_k^o M_ijo;
    # each stage uses up the previous one's values as it forms its own
    T3 = Tensor("T", (3, 3, 3, 3))
    M3 = Tensor("M", (3, 3, 3, 3))
    out.append(Program("contract3", "A_ijkl = D_k^o C_j^n B_i^m E_mnol (Sec. 5.1, "
                                    "eq:Contract3)")
               .temp(T3, M3).fuse(l).input_order(Dm, C, B, E)
               .let(T3[i, n_, o_, l], Sum(m, B[i, m] * E[m, n_, o_, l]))
               .let(M3[i, j, o_, l], Sum(n_, C[j, n_] * T3[i, n_, o_, l]))
               .let(A4[i, j, k, l], Sum(o_, Dm[k, o_] * M3[i, j, o_, l])))

    # the examples of Sec. 4 (dimension-4 indices a, b, c; fixed and offset indices)
    A = Tensor("A", (4, 4))
    Bm = Tensor("B", (4, 4))
    C = Tensor("C", (4, 4), sym=[(0, 1)])
    out.append(Program("lst_sym_contract", "C_(ab) = sum_c A_ac B_cb, symmetric left-hand "
                                           "side (Sec. 4, rank 2 contraction example)")
               .let(C[a, b], Sum(c, A[a, c] * Bm[c, b])))
    D = Tensor("D", (4, 4), sym=[(0, 1)])
    E4 = Tensor("E", (4, 4))
    F = Tensor("F", (4, 4))
    out.append(Program("lst_fixed_offset", "D_(i0) = sum_c E_(i+1)c F_c0, fixed and offset "
                                           "indices (Sec. 4, second contraction example)")
               .let(D[i, 0], Sum(c, E4[i + 1, c] * F[c, 0])))

    # spacetime split (Sec. 2.2): g_ij = psi_(i+1)(j+1), beta_i = psi_(i+1)0
    psi = Tensor("psi", (4, 4), sym=[(0, 1)])
    gs = Tensor("g", (3, 3), sym=[(0, 1)])
    bs = Tensor("beta", (3,))
    out.append(Program("spacetime_split", "spatial metric and shift from the spacetime "
                                          "metric psi_ab (Sec. 2.2)")
               .let(gs[i, j], psi[i + 1, j + 1])
               .let(bs[i], psi[i + 1, 0]))
    return out
