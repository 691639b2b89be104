"""Closed-form test fields with known Christoffel symbols, covariant
derivatives and metric evolution.

Nothing here calls the oracle or the GPU library: each function evaluates a
textbook metric (or a flat metric in curved coordinates) and its analytically
known connection, so the oracle can be pinned to something other than itself.
Field layouts follow the library's conventions:

  g, K, dtg  [6]  symmetric pair index s(i,j): 00 01 02 11 12 22
  dg        [18]  k*6 + s(i,j)   = d_k g_ij
  gamma27   [27]  (i*3+j)*3 + k  = Gamma^i_jk
  beta       [3]  i
  dbeta      [9]  j*3 + i        = d_j beta_i
  nabla      [9]  j*3 + i        = nabla_j beta_i
"""
from __future__ import annotations

import numpy as np

S = np.array([[0, 1, 2], [1, 3, 4], [2, 4, 5]])
PAIRS = ((0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2))


def sym6(M):
    """[3,3,n] symmetric -> [6,n]."""
    return np.stack([M[i, j] for i, j in PAIRS])


def full33(f):
    """[6,n] -> [3,3,n]."""
    return np.stack([np.stack([f[S[i, j]] for j in range(3)]) for i in range(3)])


def dg18(D):
    """[3(k),3,3,n] with D[k,i,j] = d_k g_ij -> [18,n]."""
    return np.concatenate([sym6(D[k]) for k in range(3)])


def dg_full(dg):
    """[18,n] -> [3(k),3,3,n]."""
    return np.stack([full33(dg[6 * k:6 * k + 6]) for k in range(3)])


def g27(Gam):
    """[3,3,3,n] Gamma[i,j,k] -> [27,n]."""
    return Gam.reshape(27, -1)


def flat_spherical(r, th):
    """Flat space in spherical coordinates (r, theta, phi)."""
    n = r.size
    s, c = np.sin(th), np.cos(th)
    g = np.zeros((3, 3, n))
    g[0, 0] = 1.0
    g[1, 1] = r * r
    g[2, 2] = r * r * s * s
    D = np.zeros((3, 3, 3, n))
    D[0, 1, 1] = 2 * r
    D[0, 2, 2] = 2 * r * s * s
    D[1, 2, 2] = 2 * r * r * s * c
    Gam = np.zeros((3, 3, 3, n))
    Gam[0, 1, 1] = -r
    Gam[0, 2, 2] = -r * s * s
    Gam[1, 0, 1] = Gam[1, 1, 0] = 1 / r
    Gam[1, 2, 2] = -s * c
    Gam[2, 0, 2] = Gam[2, 2, 0] = 1 / r
    Gam[2, 1, 2] = Gam[2, 2, 1] = c / s
    return sym6(g), dg18(D), g27(Gam)


def spherical_shift_dz(r, th):
    """The covector dz = d(r cos theta) in spherical coordinates: a gradient,
    so its covariant derivative vanishes in flat space."""
    n = r.size
    s, c = np.sin(th), np.cos(th)
    beta = np.stack([c, -r * s, np.zeros(n)])
    db = np.zeros((3, 3, n))          # db[j, i] = d_j beta_i
    db[1, 0] = -s
    db[0, 1] = -s
    db[1, 1] = -r * c
    return beta, db.reshape(9, n)


def spherical_shift_rdr(r, th):
    """The covector r dr = d(r^2/2): a homothety, nabla_j beta_i = g_ij."""
    n = r.size
    beta = np.stack([r, np.zeros(n), np.zeros(n)])
    db = np.zeros((3, 3, n))
    db[0, 0] = 1.0
    return beta, db.reshape(9, n)


def schwarzschild_areal(r, th, M):
    """Spatial Schwarzschild metric in areal coordinates (r, theta, phi)."""
    n = r.size
    s, c = np.sin(th), np.cos(th)
    f = 1 - 2 * M / r
    g = np.zeros((3, 3, n))
    g[0, 0] = 1 / f
    g[1, 1] = r * r
    g[2, 2] = r * r * s * s
    D = np.zeros((3, 3, 3, n))
    D[0, 0, 0] = -2 * M / (r * r * f * f)
    D[0, 1, 1] = 2 * r
    D[0, 2, 2] = 2 * r * s * s
    D[1, 2, 2] = 2 * r * r * s * c
    Gam = np.zeros((3, 3, 3, n))
    Gam[0, 0, 0] = -M / (r * (r - 2 * M))
    Gam[0, 1, 1] = -(r - 2 * M)
    Gam[0, 2, 2] = -(r - 2 * M) * s * s
    Gam[1, 0, 1] = Gam[1, 1, 0] = 1 / r
    Gam[1, 2, 2] = -s * c
    Gam[2, 0, 2] = Gam[2, 2, 0] = 1 / r
    Gam[2, 1, 2] = Gam[2, 2, 1] = c / s
    return sym6(g), dg18(D), g27(Gam)


def schwarzschild_isotropic(x, M):
    """Conformally flat g = psi^4 delta, psi = 1 + M/(2r), Cartesian x [3,n]."""
    n = x.shape[1]
    r = np.sqrt((x * x).sum(0))
    psi = 1 + M / (2 * r)
    dpsi = -M * x / (2 * r ** 3)            # d_k psi
    dlnpsi = dpsi / psi
    eye = np.eye(3)
    g = psi ** 4 * eye[:, :, None] * np.ones(n)
    D = 4 * psi ** 3 * dpsi[:, None, None, :] * eye[None, :, :, None]
    Gam = 2 * (eye[:, :, None, None] * dlnpsi[None, None, :, :]
               + eye[:, None, :, None] * dlnpsi[None, :, None, :]
               - eye[None, :, :, None] * dlnpsi[:, None, None, :])
    return sym6(g), dg18(D), g27(Gam)


class Curvilinear:
    """Flat space in the coordinates x of the map X(x) = x + eps q(x),
    q^a = 1/2 Q^a_ij x^i x^j (Q^a symmetric).  All 18 Christoffel symbols are
    non-zero: Gamma^k_ij = (J^-1)^k_a H^a_ij, J^a_i = dX^a/dx^i, H^a_ij =
    d_i d_j X^a.  Three shifts with known covariant derivatives: a gradient
    (nabla beta = 0), a homothety (nabla_j beta_i = g_ij) and a rotation Killing
    covector (nabla_j beta_i = J^a_i Omega_ab J^b_j, antisymmetric)."""

    def __init__(self, n, seed=7, eps=0.125):
        rng = np.random.default_rng(seed)
        x = rng.uniform(-1, 1, size=(3, n))
        x /= np.maximum(1.0, np.sqrt((x * x).sum(0)))
        Q = rng.uniform(-1, 1, size=(3, 3, 3))
        Q = 0.5 * (Q + Q.transpose(0, 2, 1))
        self.n, self.x = n, x
        self.X = x + eps * 0.5 * np.einsum("aij,in,jn->an", Q, x, x)
        self.J = np.eye(3)[:, :, None] + eps * np.einsum("aij,jn->ain", Q, x)  # J[a,i]
        self.H = eps * Q[:, :, :, None] * np.ones(n)                              # H[a,i,j]
        G = np.einsum("ain,ajn->ijn", self.J, self.J)
        D = (np.einsum("akin,ajn->kijn", self.H, self.J)
             + np.einsum("ain,akjn->kijn", self.J, self.H))
        Jinv = np.linalg.inv(self.J.transpose(2, 0, 1))                        # [n, i, a]
        Gam = np.einsum("nka,aijn->kijn", Jinv, self.H)
        self.g, self.dg, self.gamma27 = sym6(G), dg18(D), g27(Gam)
        self.gfull = G
        self.c = rng.uniform(-1, 1, size=3)
        Om = rng.uniform(-1, 1, size=(3, 3))
        self.Omega = Om - Om.T

    def gradient_shift(self):
        beta = np.einsum("a,ain->in", self.c, self.J)
        db = np.einsum("a,aijn->jin", self.c, self.H)      # d_j beta_i
        return beta, db.reshape(9, self.n)

    def homothety_shift(self):
        beta = np.einsum("an,ain->in", self.X, self.J)
        db = (np.einsum("ajn,ain->jin", self.J, self.J)
              + np.einsum("an,aijn->jin", self.X, self.H))
        return beta, db.reshape(9, self.n)

    def killing_shift(self):
        OX = np.einsum("ab,bn->an", self.Omega, self.X)
        beta = np.einsum("ain,an->in", self.J, OX)
        db = (np.einsum("aijn,an->jin", self.H, OX)
              + np.einsum("ain,ab,bjn->jin", self.J, self.Omega, self.J))
        nabla = np.einsum("ain,ab,bjn->jin", self.J, self.Omega, self.J)
        return beta, db.reshape(9, self.n), nabla.reshape(9, self.n)
