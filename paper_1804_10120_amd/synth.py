"""Seeded synthetic input fields (no arithmetic of the method lives here).

Both the GPU path's tests/benchmark and the CPU oracle are fed from these
generators, so the two sides see identical bits.  The paper runs its
benchmarks on synthetic grids of varying size with unspecified values
(Sec. 5.1); the distributions below stand in for them:

  g_ij   = delta_ij + 0.1 S_ij, the 6 stored entries of S i.i.d. U[-1,1]
           (Gershgorin: eigenvalues in [0.7, 1.3], so g is SPD, cond <= 1.86)
  d_k g_ij   U[-1,1]   (18 components)
  beta_i     U[-0.5,0.5] (3)
  d_j beta_i N(0,1)    (9)
  K_ij       U[-1,1]   (6)
  alpha      U[0.5,1.5] (1)
  W_ij       N(0,1)    (6)  -- cotangent of d_t g_ij for the adjoint

Every field is a numpy float64 array of shape [C, n] (alpha is [1, n]).  One
``numpy.random.Generator(PCG64)`` per field, spawned from
``SeedSequence(seed)`` in the fixed order g, dg, beta, dbeta, K, alpha, W, so a
field does not change when another one is added or resized.
"""
from __future__ import annotations

import numpy as np

FIELD_ORDER = ("g", "dg", "beta", "dbeta", "K", "alpha", "W")
NCOMP = {"g": 6, "dg": 18, "beta": 3, "dbeta": 9, "K": 6, "alpha": 1, "W": 6,
         "ginv": 6, "gamma": 18, "nabla": 9, "dtg": 6}
DIAG = (0, 3, 5)  # stored slots of the diagonal (00, 11, 22)

BASE_SEED = 180410120


def config_seed(config: int) -> int:
    """Seed of the workload with the given configuration number."""
    return BASE_SEED + int(config)


def make_fields(n: int, seed: int = BASE_SEED, fields=FIELD_ORDER) -> dict:
    """Seeded input fields over ``n`` grid points (see module docstring)."""
    n = int(n)
    gens = dict(zip(FIELD_ORDER,
                    (np.random.Generator(np.random.PCG64(s))
                     for s in np.random.SeedSequence(seed).spawn(len(FIELD_ORDER)))))
    out = {}
    for name in fields:
        rng = gens[name]
        if name == "g":
            a = 0.1 * rng.uniform(-1.0, 1.0, size=(6, n))
            a[list(DIAG)] += 1.0
        elif name == "dg":
            a = rng.uniform(-1.0, 1.0, size=(18, n))
        elif name == "beta":
            a = rng.uniform(-0.5, 0.5, size=(3, n))
        elif name == "dbeta":
            a = rng.standard_normal(size=(9, n))
        elif name == "K":
            a = rng.uniform(-1.0, 1.0, size=(6, n))
        elif name == "alpha":
            a = rng.uniform(0.5, 1.5, size=(1, n))
        elif name == "W":
            a = rng.standard_normal(size=(6, n))
        else:
            raise KeyError(name)
        out[name] = np.ascontiguousarray(a)
    return out


def domain_edges(ndom: int = 256, lo: int = 8, hi: int = 48, seed: int = BASE_SEED + 3):
    """Edge lengths of ``ndom`` cubic subgrids, i.i.d. uniform on the integers
    lo..hi; subgrid d has edges[d]**3 points."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    return rng.integers(lo, hi + 1, size=ndom)


# Component counts of the right-hand-side tensors of the Sec. 5.1 benchmark
# expressions, in the order they are written.
EXPR_INPUTS = {"assign1": (3,), "assign2": (9,), "assign3": (27,), "add1": (3, 3),
               "add2": (3, 3, 3), "add3": (3, 3, 3, 3), "mult1": (3, 3), "mult2": (3, 3, 3),
               "mult3": (3, 3, 3, 3), "contract1": (9, 81), "contract2": (9, 9, 81),
               "contract3": (9, 9, 9, 81), "kij": (1, 6, 3)}


def make_expr_inputs(name, n, seed=BASE_SEED):
    """Seeded inputs of benchmark expression ``name``: every tensor component
    i.i.d. U[-1,1], except the lapse of K_ij (U[0.5,1.5]).  One generator per
    input, spawned from ``SeedSequence(seed)``."""
    comps = EXPR_INPUTS[name]
    seqs = np.random.SeedSequence(seed).spawn(len(comps))
    out = []
    for k, (c, sq) in enumerate(zip(comps, seqs)):
        rng = np.random.Generator(np.random.PCG64(sq))
        lo, hi = (0.5, 1.5) if (name == "kij" and k == 0) else (-1.0, 1.0)
        out.append(np.ascontiguousarray(rng.uniform(lo, hi, size=(c, int(n)))))
    return out
