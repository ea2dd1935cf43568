"""Seeded inputs shared by the oracle pins and the GPU parity tests (input
generation only: no arithmetic of the scheme)."""
import math

import numpy as np

from paper_2412_06546_amd import cases


def fallback_case():
    """A cold gas (T = 0.08) with a velocity wave of amplitude 2 on a
    periodic triangle mesh (100 cells, 20 x 20 velocities): the limiter
    bounds each conservative variable separately, so at about a quarter of
    the cells the reconstructed kinetic energy at a face exceeds the total
    energy and the macroscopic reconstruction falls back to first order."""
    mesh = cases.periodic_triangles(10, 5, 2.0, 1.0, seed=7)
    nc = len(mesh["cell_volume"])
    x = mesh["cell_centroid"]
    prim0 = np.stack([np.ones(nc), 2.0 * np.sin(math.pi * x[:, 0]), np.zeros(nc), np.full(nc, 0.08)], 1)
    vg = cases.tensor_vgrid(20, 4.0, 2)
    gas = cases.gas_params(2 / 3, 0.81, cases.vhs_mu_ref(0.1, 0.81, 1.0), dim=2)
    return dict(name="cold_wave_fallback_100_v20x20", mesh=mesh, vgrid=vg, gas=gas, prim0=prim0)
