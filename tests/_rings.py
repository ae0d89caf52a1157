"""Seeded random rings for parity tests beyond the SPS-like ring: circumference
100 m to 30 km, harmonic 1 to 40000, protons, electrons or fully stripped
lead ions from gamma 1.5 to 2000, transition gamma 2 to 60 (above and below
transition), and a voltage whose sign makes z = 0 stable and whose size puts
the small-amplitude synchrotron tune between 5e-4 and 5e-2 (set through the
oracle's derived constants). Test infrastructure: the oracle sets the inputs,
nothing here is compared."""
import math

import numpy as np

import oracle

SPECIES = [  # (rest energy [eV], charge [e])
    (938.272e6, 1.0),      # proton
    (0.51099895e6, -1.0),  # electron
    (193.687e9, 82.0),     # Pb-208 82+
]


def random_ring(seed):
    rng = np.random.default_rng(5000 + seed)
    while True:
        mass, charge = SPECIES[int(rng.integers(len(SPECIES)))]
        gamma = 10.0 ** rng.uniform(math.log10(1.5), math.log10(2000.0))
        gamma_t = 10.0 ** rng.uniform(math.log10(2.0), math.log10(60.0))
        # keep away from transition, where the slip factor vanishes
        if abs(1.0 / gamma_t ** 2 - 1.0 / gamma ** 2) < 1e-4:
            continue
        ring = dict(circumference_m=10.0 ** rng.uniform(2.0, math.log10(3e4)),
                    harmonic=float(rng.integers(1, 40001)),
                    voltage_V=1e6, p0c_eV=mass * math.sqrt(gamma ** 2 - 1.0), mass_eV=mass,
                    gamma_t=gamma_t, charge_e=charge)
        d = oracle.derive(ring)
        if d["A"] * d["k"] * d["D"] <= 0.0:  # z = 0 unstable: the other sign of V
            ring["voltage_V"] = -ring["voltage_V"]
            d = oracle.derive(ring)
        q_target = 10.0 ** rng.uniform(math.log10(5e-4), math.log10(5e-2))
        ring["voltage_V"] *= (q_target / d["Qs"]) ** 2
        return ring


def matched_bunch(ring, n, seed, fill=0.25):
    """Gaussian bunch with sigma_dp = fill x the bucket half-height and the
    linearly matched sigma_z."""
    d = oracle.derive(ring)
    sigma_dp = fill * d["bucket_height"]
    sigma_z = sigma_dp * abs(d["D"]) / d["omega"]
    rng = np.random.default_rng(7000 + seed)
    return rng.normal(0.0, sigma_z, n), rng.normal(0.0, sigma_dp, n)
