"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle runs.

This module holds workload recipes only (random draws, ring parameter sets,
the FP32 hi/compensation encoding of an FP64 array). It contains none of the
tracking arithmetic and imports neither the oracle nor the HIP package.

The paper tracks macro-particles read from two-column (z, delta) data files
written by a Python script (section 2.2); it does not state the distribution.
These generators stand in for those files: Gaussian bunches drawn with NumPy's
PCG64 from fixed seeds.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

# Single-harmonic proton ring used by the plain, paper-scale and precision
# workloads: C = 6911 m, h = 4620, V = 2 MV, p0 c = 26 GeV, m c^2 = 0.938 GeV,
# gamma_t = 22.77, charge +1 e.
SPS_RING = dict(circumference_m=6911.0, harmonic=4620.0, voltage_V=2.0e6,
                p0c_eV=26.0e9, mass_eV=0.938e9, gamma_t=22.77, charge_e=1.0)

# Extended-map workload: the same ring with a second RF system at twice the
# harmonic and a quarter of the voltage in counter-phase (bunch-lengthening
# double RF), and slip factor eta0 + eta1 dp + eta2 dp^2 with eta0 ~ 6.29e-4
# the ring's own value at 26 GeV.
SPS_DOUBLE_RF = dict(SPS_RING, phi1_rad=0.0, harmonic2=9240.0, voltage2_V=0.5e6,
                     phi2_rad=math.pi, eta1=2.5e-4, eta2=-1.9e-2)

# Transverse optics of the 6-D workload at the observation point: SPS-like
# tunes, chromaticities (tune shift per unit dp) and Twiss parameters (m).
SPS_TWISS = dict(q_x=20.13, qp_x=1.5, alpha_x=0.7, beta_x=42.0,
                 q_y=20.18, qp_y=-2.5, alpha_y=-1.1, beta_y=87.0)

# Longitudinal wake of the wake workload: a broadband resonator (10 kOhm,
# 1 GHz, Q = 1) on a bunch of 1e11 protons, 256 slices over +-0.8 m.
SPS_WAKE = dict(model="resonator", n_slices=256, shunt=1e4, freq_hz=1.0e9, quality=1.0,
                intensity=1e11, z_lo=-0.8, z_hi=0.8)

SIGMA_Z = 0.23      # metres
SIGMA_DP = 1.0e-3   # relative momentum deviation

# Seeds per workload (1001: 1e3 particles x 1e3 turns; 1002: 1e6 x 1e4;
# 1003: 1e7 x 1e5; 1004: 256 uneven bunches; 1005: request stream).
SEEDS = {"small": 1001, "paper_scale": 1002, "precision": 1003, "batched": 1004,
         "serving": 1005}


def gaussian_bunch(n: int, sigma_z: float, sigma_dp: float, seed: int):
    """z ~ N(0, sigma_z), dp ~ N(0, sigma_dp), independent, FP64, PCG64(seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    z = rng.standard_normal(n) * sigma_z
    dp = rng.standard_normal(n) * sigma_dp
    return z, dp


def split_f32c(x):
    """Encode FP64 values as an FP32 pair (hi, comp) with value = hi - comp.

    hi is x rounded to FP32 and comp = fl32(hi - x) holds the rounding error,
    so hi - comp reproduces x to about 2^-48 relative.
    """
    x = np.asarray(x, dtype=np.float64)
    hi = x.astype(np.float32)
    comp = (hi.astype(np.float64) - x).astype(np.float32)
    return hi, comp


def join_f32c(hi, comp):
    """The FP64 value an (hi, comp) pair stands for: hi - comp, exact in FP64."""
    return np.asarray(hi, dtype=np.float64) - np.asarray(comp, dtype=np.float64)


@dataclass
class BunchSpec:
    n: int
    voltage_V: float
    harmonic: float
    sigma_dp: float
    seed: int


def batched_specs(seed: int = SEEDS["batched"], n_bunches: int = 256,
                  log10_n=(3.0, 6.0)):
    """Bunch table for the uneven batched workload: n_b = round(10^U(3,6)),
    V_b ~ U[1, 8] MV, h_b uniform over {4620, 9240}, sigma_dp ~ U[5e-4, 2e-3].
    Each bunch gets its own particle seed (seed * 1000 + index)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    specs = []
    for b in range(n_bunches):
        n = int(round(10.0 ** rng.uniform(*log10_n)))
        v = float(rng.uniform(1.0e6, 8.0e6))
        h = 4620.0 if rng.integers(0, 2) == 0 else 9240.0
        sd = float(rng.uniform(5.0e-4, 2.0e-3))
        specs.append(BunchSpec(n=n, voltage_V=v, harmonic=h, sigma_dp=sd,
                               seed=seed * 1000 + b))
    return specs


def ring_for(spec: BunchSpec) -> dict:
    """The ring of a batched/served bunch: the base ring with its own V and h."""
    r = dict(SPS_RING)
    r["voltage_V"] = spec.voltage_V
    r["harmonic"] = spec.harmonic
    return r


@dataclass
class RequestSpec:
    rid: int
    arrival_s: float
    n: int
    turns: int
    integrator: str
    dtype: str
    voltage_V: float
    harmonic: float
    sigma_dp: float
    seed: int


def request_stream(rate_hz: float, count: int, seed: int = SEEDS["serving"],
                   log10_n=(3.0, 7.0), log10_turns=(3.0, 5.0)):
    """Poisson arrivals at ``rate_hz``; each request draws n = round(10^U(3,7)),
    turns = round(10^U(3,5)), an integrator from {euler_cromer, leapfrog,
    ruth4}, a dtype from {f64, f32c}, V ~ U[1, 8] MV, h from {4620, 9240} and
    sigma_dp ~ U[5e-4, 2e-3]. The particle seed of request i is 10^6 + i."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    for i in range(count):
        t += float(rng.exponential(1.0 / rate_hz)) if rate_hz > 0 else 0.0
        n = int(round(10.0 ** rng.uniform(*log10_n)))
        turns = int(round(10.0 ** rng.uniform(*log10_turns)))
        integ = ("euler_cromer", "leapfrog", "ruth4")[int(rng.integers(0, 3))]
        dt = ("f64", "f32c")[int(rng.integers(0, 2))]
        v = float(rng.uniform(1.0e6, 8.0e6))
        h = 4620.0 if rng.integers(0, 2) == 0 else 9240.0
        sd = float(rng.uniform(5.0e-4, 2.0e-3))
        out.append(RequestSpec(rid=i, arrival_s=t, n=n, turns=turns, integrator=integ,
                               dtype=dt, voltage_V=v, harmonic=h, sigma_dp=sd,
                               seed=1_000_000 + i))
    return out


def log_uniform_mean(lo_exp: float, hi_exp: float) -> float:
    """E[10^U(lo, hi)] for sizing estimates."""
    a, b = 10.0 ** lo_exp, 10.0 ** hi_exp
    return (b - a) / (math.log(10.0) * (hi_exp - lo_exp))
