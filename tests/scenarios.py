"""Seeded synthetic scenarios shared by the oracle pins and the GPU parity
tests (parameters and input beams only; no step arithmetic)."""
from __future__ import annotations

import numpy as np

from paper_1612_07592_amd import workloads as W


def base(**kw):
    d = dict(cfl=0.95, lambda_m=1e-6, duration_cycles=10.0, photon_cut_mc2=0.0, ncs=True,
             brem=True, frozen=False, no_recoil=False, seed=7, job_id=0, w0_lambda=0.0,
             focus_x_lambda=0.0, precision="fp64", photon_capacity=1 << 20, a0=0.0,
             Z=13, charge_state=13, ne_over_nc=50.0)
    d.update(kw)
    return d


def frozen_B_beam(n_cells=1024, ppc=64, slab=(480, 544), B=1000.0, ne=50.0, **kw):
    """Particle-only mode, uniform B along z; electrons get random-direction
    momenta (set with beam_momenta) and gyrate inside the box."""
    dx = 1 / 128
    return base(name="frozen-B", dims=1, n=[n_cells], dx_lambda=[dx], ppc=ppc,
                x0_lambda=slab[0] * dx, thickness_lambda=(slab[1] - slab[0]) * dx,
                frozen=True, frozen_kind=0, frozen_E=[0.0, 0.0, 0.0], frozen_B=[0.0, 0.0, B],
                ne_over_nc=ne, **kw)


def beam_momenta(n, pmin, pmax, seed, planar=True):
    """Log-uniform |p| in [pmin, pmax], isotropic direction (in the x-y plane
    when planar)."""
    rng = np.random.default_rng(seed)
    pm = np.exp(rng.uniform(np.log(pmin), np.log(pmax), n))
    if planar:
        th = rng.uniform(0, 2 * np.pi, n)
        d = np.stack([np.cos(th), np.sin(th), np.zeros(n)], axis=1)
    else:
        v = rng.normal(size=(n, 3))
        d = v / np.linalg.norm(v, axis=1, keepdims=True)
    return d * pm[:, None]


def frozen_plane_wave(a=50.0, **kw):
    dx = 1 / 128
    return base(name="frozen-pw", dims=1, n=[2048], dx_lambda=[dx], ppc=32, x0_lambda=1.0,
                thickness_lambda=1.0, frozen=True, frozen_kind=1, frozen_a=a, **kw)


def c1_parity(steps=256):
    w = W.c1(steps)
    w["photon_cut_mc2"] = 0.0   # every NCS event leaves a record, so lists compare 1:1
    return w


def small_2d(steps=160, a0=60.0, precision="fp64"):
    return base(name="small-2d", dims=2, n=[128, 64], dx_lambda=[1 / 32, 1 / 32], ppc=4,
                x0_lambda=1.0, thickness_lambda=0.5, a0=a0, w0_lambda=0.8,
                focus_x_lambda=1.0, steps=steps, precision=precision, Z=79, charge_state=69,
                ne_over_nc=40.0, seed=3)


def small_3d(steps=80, a0=60.0, precision="fp64"):
    return base(name="small-3d", dims=3, n=[40, 16, 16], dx_lambda=[1 / 16, 1 / 16, 1 / 16],
                ppc=2, x0_lambda=1.0, thickness_lambda=0.5, a0=a0, w0_lambda=0.4,
                focus_x_lambda=1.0, steps=steps, precision=precision, Z=79, charge_state=69,
                ne_over_nc=40.0, seed=4)


def ions_1d(steps=300, precision="fp64"):
    """1D laser-slab run with mobile ions light enough (q/M = 0.016) to move
    within the run, in a dense gold-like slab."""
    dx = 1 / 128
    return base(name="ions-1d", dims=1, n=[1024], dx_lambda=[dx], ppc=32, ion_ppc=8,
                ion_mass_me=5000.0, x0_lambda=0.25, thickness_lambda=1.0, a0=270.0,
                duration_cycles=3.0, envelope="flat", steps=steps, precision=precision,
                Z=79, charge_state=79, ne_over_nc=400.0, seed=41)


def ions_2d(steps=160, precision="fp64"):
    """2D laser-slab run with mobile ions, flat envelope."""
    return base(name="ions-2d", dims=2, n=[128, 64], dx_lambda=[1 / 32, 1 / 32], ppc=4,
                ion_ppc=2, ion_mass_me=2000.0, x0_lambda=1.0, thickness_lambda=0.5, a0=120.0,
                w0_lambda=0.8, focus_x_lambda=1.0, duration_cycles=2.0, envelope="flat",
                steps=steps, precision=precision, Z=79, charge_state=79, ne_over_nc=60.0,
                seed=43)


def frozen_dense_ions(B=50.0, steps=150):
    """Particle-only mode at a very high density with mobile ions gyrating in
    a uniform B: many bremsstrahlung events, each decided against the counted
    ion density of the electron's cell."""
    return frozen_B_beam(B=B, ne=5e7, Z=79, charge_state=79, ion_ppc=4, ion_mass_me=200.0,
                         steps=steps)


def ions_3d(steps=80, precision="fp64"):
    """3D laser-slab run with mobile ions (small box, several tiles)."""
    return base(name="ions-3d", dims=3, n=[64, 16, 16], dx_lambda=[1 / 16, 1 / 16, 1 / 16], ppc=2,
                ion_ppc=1, ion_mass_me=1000.0, x0_lambda=1.0, thickness_lambda=0.5, a0=150.0,
                w0_lambda=0.6, focus_x_lambda=1.0, duration_cycles=2.0, envelope="flat",
                steps=steps, precision=precision, Z=79, charge_state=79, ne_over_nc=30.0, seed=45)
