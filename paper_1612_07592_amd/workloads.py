"""Workload recipes: the synthetic inputs of every configuration, as data.

This module holds parameters only (no step arithmetic) and imports nothing
from the rest of the package, so both the HIP path and the CPU oracle can be
driven from the same recipe.  Every input is synthetic and seeded: electrons
are loaded cold (p = 0) at uniform-random in-cell positions drawn from the
run's own Philox stream, the ions have n_i = n_e / charge_state (static, or
mobile macro-ions loaded the same way at rest),
and the laser enters from the left boundary (Sec. III of the paper sets up the
same geometry: linear polarisation along y, propagation along x, a slab target
of Al or Au).

Keys (lengths in laser wavelengths, lambda = 1 um):
  dims, n (cells per axis), dx_lambda, cfl, steps, ppc (electrons per cell),
  Z, charge_state, ne_over_nc, x0_lambda (slab front), thickness_lambda,
  a0, w0_lambda (0 = plane wave), duration_cycles (sin^2 envelope, full
  length), focus_x_lambda, photon_cut_mc2 (NCS record cut; Sec. III keeps
  photons of at least m_e c^2), ncs, brem, frozen (particle-only mode),
  frozen_kind/frozen_E/frozen_B/frozen_a, seed, job_id, photon_capacity,
  precision ("fp64" or "fp32"), ion_ppc (mobile ions per slab cell, 0 =
  static), ion_mass_me, envelope ("sin2" or "flat").
"""
from __future__ import annotations

import math
import random

AL = dict(Z=13, charge_state=13, ne_over_nc=50.0)
AU = dict(Z=79, charge_state=69, ne_over_nc=200.0)


def _base(**kw):
    d = dict(cfl=0.95, lambda_m=1e-6, duration_cycles=10.0, photon_cut_mc2=1.0,
             ncs=True, brem=True, frozen=False, no_recoil=False, seed=1, job_id=0,
             w0_lambda=0.0, focus_x_lambda=0.0, precision="fp64")
    d.update(kw)
    return d


def c1(steps=256):
    """1D3V FP64: 1024 cells over 8 um, Al slab 1 um at n_e = 50 n_c, 64/cell,
    plane wave a0 = 27, 256 steps.  The slab front sits at 0.25 um so that
    the pulse reaches it within the run."""
    return _base(name="C1-1d-al-a27", dims=1, n=[1024], dx_lambda=[1 / 128], ppc=64,
                 x0_lambda=0.25, thickness_lambda=1.0, a0=27.0, steps=steps, seed=1,
                 photon_capacity=1 << 20, **AL)


def c2(steps=2000, precision="fp32"):
    """2D3V: 2048x1024 cells at lambda/64, Au (q = 69) slab 2 um thick at
    x = 2 um, n_e = 200 n_c, 16/cell, Gaussian w0 = 3 um focused on the slab
    front, a0 = 270."""
    return _base(name="C2-2d-au-a270", dims=2, n=[2048, 1024], dx_lambda=[1 / 64, 1 / 64],
                 ppc=16, x0_lambda=2.0, thickness_lambda=2.0, a0=270.0, w0_lambda=3.0,
                 focus_x_lambda=2.0, steps=steps, seed=2, photon_capacity=400_000_000,
                 precision=precision, **AU)


def c3_jobs(steps=1000):
    """Intensity x target scan: a0 in {27, 85, 270, 854} x {Al, Au}, 2D3V."""
    grids = {27.0: (512, 256), 85.0: (1024, 512), 270.0: (1024, 512), 854.0: (2048, 1024)}
    jobs = []
    j = 0
    for a0 in (27.0, 85.0, 270.0, 854.0):
        for tgt, thick, ppc in ((AL, 1.0, 8), (AU, 2.0, 16)):
            nx, ny = grids[a0]
            jobs.append(_base(name=f"C3-{j}", dims=2, n=[nx, ny], dx_lambda=[1 / 64, 1 / 64],
                              ppc=ppc, x0_lambda=2.0, thickness_lambda=thick, a0=a0,
                              w0_lambda=3.0, focus_x_lambda=2.0, steps=steps, seed=10 + j,
                              job_id=j, photon_capacity=50_000_000, precision="fp32", **tgt))
            j += 1
    return jobs


def c4_stream(n_jobs=500, rate_per_s=4.0, seed=2026, max_electrons=3e7):
    """Poisson arrivals of scan jobs (1D3V or 2D3V).  Returns (arrival_s, job)."""
    rng = random.Random(seed)
    t = 0.0
    out = []
    for k in range(n_jobs):
        t += rng.expovariate(rate_per_s)
        dims = 1 if rng.random() < 0.5 else 2
        a0 = math.exp(rng.uniform(math.log(27.0), math.log(854.0)))
        tgt = AL if rng.random() < 0.5 else AU
        thick = rng.uniform(0.5, 4.0)
        ne_target = math.exp(rng.uniform(math.log(1e5), math.log(max_electrons)))
        steps = rng.randint(200, 2000)
        dx = 1 / 64
        slab = max(1, round(thick / dx))
        nx = 1024 if thick < 3.0 else 1536
        if dims == 1:
            ppc = max(1, round(ne_target / slab))
            job = _base(name=f"C4-{k}", dims=1, n=[nx], dx_lambda=[dx], ppc=ppc)
        else:
            ny = max(16, int(ne_target / (slab * 16)))
            job = _base(name=f"C4-{k}", dims=2, n=[nx, ny], dx_lambda=[dx, dx], ppc=16,
                        w0_lambda=3.0)
        job.update(x0_lambda=2.0, thickness_lambda=thick, a0=a0, focus_x_lambda=2.0,
                   steps=steps, seed=1000 + k, job_id=k, photon_capacity=20_000_000,
                   precision="fp32", **tgt)
        out.append((t, job))
    return out


def c5(steps=500):
    """3D3V: 512x256x256 cells at lambda/32, Au (q = 69) slab 1 um at x = 2 um,
    n_e = 200 n_c, 64 electrons per cell (4 per axis; 1.34e8 electrons),
    a0 = 854, w0 = 3 um, photon buffer for 2e8 macrophotons."""
    return _base(name="C5-3d-au-a854", dims=3, n=[512, 256, 256],
                 dx_lambda=[1 / 32, 1 / 32, 1 / 32], ppc=64, x0_lambda=2.0,
                 thickness_lambda=1.0, a0=854.0, w0_lambda=3.0, focus_x_lambda=2.0,
                 steps=steps, seed=5, photon_capacity=200_000_000, precision="fp32", **AU)


def thick_target(steps=2000, precision="fp32", energy_mev=100.0, electrons=2_097_152):
    """Particle-only thick-target run (the bremsstrahlung benchmark of Sec.
    II.B: field solve and deposit off, an electron bunch into a 5 mm gold
    target): solid gold fully ionised (n_e = 4177 n_c, Sec. III), 5000 um at
    dx = 1 um, NCS off, no fields.  `beam_energy_mev` is the kinetic energy of
    the pencil beam the caller sets along +x at the front face (all electrons
    in the first cell); the loader's uniform fill only provides the count and
    the ids.  No electron leaves the target within 5000 steps, so no sort."""
    n_cells = 5120
    thick = 5000.0
    ppc = -(-electrons // int(thick))
    return _base(name="thick-au-5mm", dims=1, n=[n_cells], dx_lambda=[1.0], ppc=ppc,
                 x0_lambda=0.0, thickness_lambda=thick, Z=79, charge_state=79,
                 ne_over_nc=4177.0, ncs=False, brem=True, frozen=True, frozen_kind=0,
                 frozen_E=[0.0, 0.0, 0.0], frozen_B=[0.0, 0.0, 0.0], steps=steps, seed=9,
                 photon_capacity=40_000_000, precision=precision, sort_every=-1,
                 beam_energy_mev=energy_mev)


# Solid targets of Sec. III: fully ionised at solid density
U_ME = 1822.888486                      # atomic mass unit in electron masses
SOLID = {
    "al": dict(Z=13, charge_state=13, ne_over_nc=711.0, ion_mass_me=26.9815385 * U_ME,
               cells=1000),
    "au": dict(Z=79, charge_state=79, ne_over_nc=4177.0, ion_mass_me=196.966569 * U_ME,
               cells=2000),
}
# peak intensities of the four runs (W/cm^2) and the a0 of a linearly
# polarised 1 um laser: a0 = 0.855 sqrt(I / 1e18 W/cm^2)
SOLID_INTENSITIES = (1e21, 1e22, 1e23, 1e24)


def a0_of_intensity(intensity_w_cm2, lambda_um=1.0):
    return 0.855 * lambda_um * math.sqrt(intensity_w_cm2 / 1e18)


def solid(target="au", intensity=1e22, process="both", cells=None, ppc=80, ion_ppc=20,
          steps=None, precision="fp32", photon_capacity=None, seed=31):
    """The laser-solid runs of Sec. III: 2D3V, a 6 x 6 um box (1000^2 cells
    for Al, 2000^2 for Au; `cells` overrides the count per axis), a fully
    ionised slab 1 um thick from x = 2 um at n_e = 711 n_c (Al) or 4177 n_c
    (Au), 80 electrons and 20 mobile ions per cell, a laser polarised along y
    with a flat 30 fs envelope and a Gaussian transverse profile of 1 um
    waist focused on the slab front, photons kept from m_e c^2 up.
    `process` = "ncs" or "brem" switches one emission off (the paper's
    separate runs), "both" keeps both.  The default run length covers the
    pulse's transit to the slab, its 30 fs and one more period."""
    t = SOLID[target]
    n = int(cells or t["cells"])
    dx = 6.0 / n
    duration = 30e-15 * 299792458.0 / 1e-6      # 30 fs in periods of a 1 um laser
    if steps is None:
        dt = 0.95 / math.sqrt(2.0 / (2 * math.pi * dx) ** 2)
        steps = int(math.ceil((duration + 2.0 + 1.0 + 1.0) * 2 * math.pi / dt))
    a0 = a0_of_intensity(intensity)
    if photon_capacity is None:
        slab = int(round(1.0 / dx)) * n
        photon_capacity = min(400_000_000, max(1 << 20, slab * ppc * 8))
    return _base(name=f"solid-{target}-I{intensity:.0e}-{process}", dims=2, n=[n, n],
                 dx_lambda=[dx, dx], ppc=ppc, ion_ppc=ion_ppc, x0_lambda=2.0,
                 thickness_lambda=1.0, a0=a0, w0_lambda=1.0, focus_x_lambda=2.0,
                 duration_cycles=duration, envelope="flat", steps=steps,
                 ncs=process in ("ncs", "both"), brem=process in ("brem", "both"),
                 photon_capacity=photon_capacity, precision=precision, seed=seed,
                 Z=t["Z"], charge_state=t["charge_state"], ne_over_nc=t["ne_over_nc"],
                 ion_mass_me=t["ion_mass_me"])


def num_electrons(w):
    """Macro-electrons the recipe loads: slab cells times ppc."""
    dx = w["dx_lambda"][0]
    i0 = int(round(w["x0_lambda"] / dx))
    i1 = i0 + int(round(w["thickness_lambda"] / dx))
    i0 = max(0, min(i0, w["n"][0]))
    i1 = max(i0, min(i1, w["n"][0]))
    cells = i1 - i0
    for a in range(1, w["dims"]):
        cells *= w["n"][a]
    return cells * w["ppc"]
