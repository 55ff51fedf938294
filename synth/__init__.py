"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only draws random numbers and describes workload shapes; it contains
none of the simulation's arithmetic (no group algebra, no Poisson solve, no field
update).  Both the CPU reference and the GPU library receive exactly these arrays.

Workload recipe (lattice units a_L = 1, coupling absorbed into the fields):
* MV colour charges (Sec. 2, Gaussian functional W[rho]): rho^a(x_T) i.i.d. normal
  with standard deviation mu / a_T per transverse site (the 2D delta function of
  the MV correlator discretised on cells of area a_T^2), one draw per colour
  component, transverse site and nucleus.
* Generic test states: normal algebra components with a chosen scale.
"""
from dataclasses import dataclass, field
import numpy as np


def rng(seed):
    return np.random.default_rng(np.random.PCG64(seed))


def mv_charges(seed, nc, nt, mu, a_T):
    """(rhoT_A, rhoT_B), each (nc^2-1, nt, nt) float64."""
    g = rng(seed)
    ng = nc * nc - 1
    sd = mu / a_T
    A = g.standard_normal((ng, nt, nt)) * sd
    B = g.standard_normal((ng, nt, nt)) * sd
    return A, B


def mv_sheet_charges(seed, nc, nt, mu, a_T, ns):
    """(rhoT_A, rhoT_B), each (ns, nc^2-1, nt, nt) float64: ns independent sheets per
    nucleus, each with variance mu^2 / ns, so that their sum has the MV variance mu^2."""
    g = rng(seed)
    ng = nc * nc - 1
    sd = mu / (a_T * np.sqrt(ns))
    A = g.standard_normal((ns, ng, nt, nt)) * sd
    B = g.standard_normal((ns, ng, nt, nt)) * sd
    return A, B


def normal(seed, shape, scale=1.0):
    return rng(seed).standard_normal(shape) * scale


def uniform(seed, shape, lo=0.0, hi=1.0):
    return rng(seed).uniform(lo, hi, shape)


@dataclass
class Workload:
    """One lattice event: sizes and physics inputs."""
    name: str
    nc: int
    nz: int
    nt: int
    a_T: float = 4.0
    a_L: float = 1.0
    dt: float = 0.5
    mu: float = 1.0
    sigma: float = 4.0
    m_ir: float = 0.2
    uv_cut: float = 0.0
    steps: int = 100
    seed: int = 1001
    zA: float = None
    zB: float = None

    def __post_init__(self):
        if self.zA is None:
            self.zA = 0.75 * self.nz * self.a_L
        if self.zB is None:
            self.zB = 0.25 * self.nz * self.a_L

    @property
    def sites(self):
        return self.nz * self.nt * self.nt


# The workloads of the method's evaluation.
SMALL_SU2 = Workload("su2-64x8x8", nc=2, nz=64, nt=8, mu=1.0, sigma=4.0, steps=100, seed=1001)
PLAIN_SU3 = Workload("su3-512x64x64", nc=3, nz=512, nt=64, mu=0.5, sigma=8.0,
                     uv_cut=2.5, steps=1024, seed=2001)
PRECISION_SU3 = Workload("su3-2048x192x192", nc=3, nz=2048, nt=192, mu=0.5, sigma=16.0,
                         uv_cut=2.5, steps=2048, seed=3001)
ADJOINT_SU3 = Workload("su3-256x32x32", nc=3, nz=256, nt=32, mu=0.5, sigma=8.0,
                       uv_cut=2.5, steps=256, seed=5001)


def batched_events(n_events=64, seed=4000):
    """64 events with N_z in {128,256,384}, N_T in {32,48,64}, mu ~ U[0.3,0.7],
    sigma ~ U[4,12], drawn from one seed; event e uses seed 4000 + e for its charges."""
    g = rng(seed)
    nzs = g.choice([128, 256, 384], size=n_events)
    nts = g.choice([32, 48, 64], size=n_events)
    mus = g.uniform(0.3, 0.7, n_events)
    sigmas = g.uniform(4.0, 12.0, n_events)
    return [Workload(f"event{e}", nc=3, nz=int(nzs[e]), nt=int(nts[e]), mu=float(mus[e]),
                     sigma=float(sigmas[e]), uv_cut=2.5, steps=512, seed=seed + e)
            for e in range(n_events)]
