"""Pins of the oracle's field side in 2D and 3D, each against something other
than the oracle itself: the exact eigenmodes of the Yee scheme, exact
reproduction of multilinear fields by the linear gather, charge continuity of
the deposit with a stated bound on the current's fixed-point rounding, the
time average of the charge along a straight path, the paraxial Gaussian beam,
and the absorbing faces.

Every check is a plain function taking the oracle library to run (None = the
oracle itself), so that tests/test_oracle_mutants.py can show that each fails
on a copy of the oracle with a planted mistake.  CPU only.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

import oracle
import scenarios as S

TWOPI = 2.0 * math.pi
ESTAG = [(1, 0, 0), (0, 1, 0), (0, 0, 1)]
BSTAG = [(0, 1, 1), (1, 0, 1), (1, 1, 0)]


def _vacuum(dims, n, dx_lambda, **kw):
    """An empty box (no electrons, no laser, no emission)."""
    d = dict(name="vacuum", dims=dims, n=list(n), dx_lambda=list(dx_lambda), ppc=1,
             x0_lambda=0.0, thickness_lambda=0.0, a0=0.0, ncs=False, brem=False)
    d.update(kw)
    return S.base(**d)


def _tables():
    import conftest
    return conftest.oracle_tables(13)


class Layout:
    """Node positions of the oracle's field arrays: index (i+g) + sx((j+g) +
    sy(k+g)), g = 2 guard cells on active axes, a staggered component sits
    half a cell up along its staggered axes."""

    def __init__(self, o, dims):
        d = o.derived()
        self.dims = dims
        self.dx = d["dx"]
        self.dt = d["dt"]
        self.n = list(o.workload["n"]) + [1] * (3 - dims)
        self.sz = [self.n[a] + 5 if a < dims else 1 for a in range(3)]
        self.g = [2 if a < dims else 0 for a in range(3)]
        self.size = self.sz[0] * self.sz[1] * self.sz[2]
        idx = np.arange(self.size)
        i = idx % self.sz[0] - self.g[0]
        j = (idx // self.sz[0]) % self.sz[1] - self.g[1]
        k = idx // (self.sz[0] * self.sz[1]) - self.g[2]
        self.ijk = np.stack([i, j, k])

    def pos(self, stag):
        return np.stack([(self.ijk[a] + 0.5 * stag[a]) * self.dx[a] if a < self.dims
                         else np.zeros(self.size) for a in range(3)])

    def interior(self, margin):
        m = np.ones(self.size, dtype=bool)
        for a in range(self.dims):
            m &= (self.ijk[a] >= margin) & (self.ijk[a] <= self.n[a] - margin)
        return m


# --------------------------------------------------------------- Yee modes
def _yee_mode(dims, n, dx_lambda, kcells, pol, steps, lib=None):
    """Largest deviation from the exact discrete plane wave after `steps`
    steps, in the interior the boundaries cannot reach.  The Yee scheme
    advances exp(i(k.x - w t)) exactly when each derivative acts as
    i K_a, K_a = 2 sin(k_a dx_a / 2) / dx_a, and 2 sin(w dt / 2) / dt = |K|;
    with E = e cos(k.x - w t) (e normal to K) and
    B = (K x e) / |K| cos(k.x - w t) at each component's own staggered node
    (B half a step behind E), every interior node follows the closed form."""
    o = oracle.OracleSim(_vacuum(dims, n, dx_lambda), _tables(), nthreads=8, lib=lib)
    L = Layout(o, dims)
    k = np.array([TWOPI / (kcells[a] * L.dx[a]) if a < dims else 0.0 for a in range(3)])
    K = np.array([2.0 * math.sin(k[a] * L.dx[a] / 2) / L.dx[a] if a < dims else 0.0
                  for a in range(3)])
    Km = np.linalg.norm(K)
    w = 2.0 / L.dt * math.asin(Km * L.dt / 2)
    e = np.asarray(pol, dtype=float)
    e = e - K * (K @ e) / Km ** 2
    e /= np.linalg.norm(e)
    b = np.cross(K, e) / Km

    def fields(t_e, t_b):
        F = np.zeros((6, L.size))
        for c in range(3):
            F[c] = e[c] * np.cos(k @ L.pos(ESTAG[c]) - w * t_e)
            F[3 + c] = b[c] * np.cos(k @ L.pos(BSTAG[c]) - w * t_b)
        return F

    o.set_fields(fields(0.0, -0.5 * L.dt))
    o.step(steps)
    ref = fields(steps * L.dt, (steps - 0.5) * L.dt)
    sel = L.interior(steps + 3)
    assert sel.sum() > 50
    err = np.abs(o.fields()[:, sel] - ref[:, sel]).max()
    o.close()
    return err


def check_yee_modes(lib=None):
    """2D (both polarisations) and 3D (two polarisations) eigenmodes, on cells
    of different sizes per axis."""
    errs = [
        _yee_mode(2, [64, 48], [1 / 16, 1 / 12], [10.0, 7.0], [0, 0, 1], 12, lib),
        _yee_mode(2, [64, 48], [1 / 16, 1 / 12], [9.0, -6.0], [1, 0, 0], 12, lib),
        _yee_mode(3, [40, 36, 32], [1 / 16, 1 / 14, 1 / 12], [9.0, 7.0, -8.0], [0, 1, 0], 10, lib),
        _yee_mode(3, [40, 36, 32], [1 / 16, 1 / 14, 1 / 12], [-8.0, 11.0, 6.0], [1, 0, 1], 10, lib),
    ]
    assert max(errs) < 1e-11, errs
    return errs


def test_yee_eigenmodes_2d_3d(oracle_lib):
    print(check_yee_modes())


# ---------------------------------------------------------------- gather
def check_gather_multilinear(lib=None):
    """Linear weights on the Yee stagger reproduce any multilinear field
    (1, x, y, z, xy, xz, yz, xyz) exactly: each component set to such a
    function of its own node positions must be gathered as that function of
    the electron position, anywhere in the box."""
    rng = np.random.default_rng(5)
    worst = 0.0
    for dims, n, dxl in ((2, [24, 20], [1 / 16, 1 / 10]), (3, [14, 12, 10], [1 / 16, 1 / 12, 1 / 10])):
        o = oracle.OracleSim(_vacuum(dims, n, dxl), _tables(), nthreads=1, lib=lib)
        L = Layout(o, dims)
        coef = rng.normal(size=(6, 8))

        def f(c, X):
            x, y, z = X
            return (coef[c, 0] + coef[c, 1] * x + coef[c, 2] * y + coef[c, 3] * z
                    + coef[c, 4] * x * y + coef[c, 5] * x * z + coef[c, 6] * y * z
                    + coef[c, 7] * x * y * z)
        F = np.zeros((6, L.size))
        for c in range(3):
            F[c] = f(c, L.pos(ESTAG[c]))
            F[3 + c] = f(3 + c, L.pos(BSTAG[c]))
        o.set_fields(F)
        for _ in range(200):
            X = np.zeros(3)
            for a in range(dims):
                X[a] = rng.uniform(1.0, n[a] - 1.0) * L.dx[a]
            for c in range(6):
                worst = max(worst, abs(o.probe_field(c, X) - f(c, X)))
        o.close()
    assert worst < 1e-12, worst
    return worst


def test_gather_reproduces_multilinear_fields(oracle_lib):
    print(check_gather_multilinear())


# ----------------------------------------------------------- continuity
def _thermal(o, sigma, seed):
    rng = np.random.default_rng(seed)
    e = o.electrons()
    return e["x"], rng.normal(scale=sigma, size=(o.N, 3)), e["tau"]


def _rho_nodes(L, x, w, alive):
    """Charge density of the electrons (charge -1, weight w) on the nodes by
    the linear weights: node (i, j, k) at (i dx, j dy, k dz)."""
    V = float(np.prod(L.dx[:L.dims]))
    r = np.zeros(L.size)
    x, w = x[alive], w[alive]
    g = [x[:, a] / L.dx[a] for a in range(L.dims)]
    c = [np.floor(ga).astype(int) for ga in g]
    f = [ga - ca for ga, ca in zip(g, c)]
    for corner in range(1 << L.dims):
        idx = np.zeros(len(w), dtype=np.int64)
        wt = -w / V
        stride = 1
        for a in range(L.dims):
            o = (corner >> a) & 1
            wt = wt * (f[a] if o else 1.0 - f[a])
            idx += (c[a] + o + L.g[a]) * stride
            stride *= L.sz[a]
        np.add.at(r, idx, wt)
    return r


def _div_E(L, F):
    """Divergence of E at the nodes: E_a is stored half a cell above its node
    along a, so dE_a/dx_a at node i is (E_a[i] - E_a[i-1]) / dx_a."""
    div = np.zeros(L.size)
    stride = 1
    for a in range(L.dims):
        Ea = F[a]
        d = np.zeros(L.size)
        d[stride:] = (Ea[stride:] - Ea[:-stride]) / L.dx[a]
        div += d
        stride *= L.sz[a]
    return div


# Fixed-point current: every contribution is rounded to the nearest multiple
# of q = 2^-40, an error of at most q/2 each.  One step changes E_a by -dt J_a,
# so div E - rho picks up at most dt * sum_a (2 / dx_a) * M * q / 2 per node and
# step, M being the most contributions one current node receives in a step
# (every electron whose deposit window holds the node: at most those of the
# 3^d cells around it... counted generously as 4^d times the electrons per cell).
def current_rounding_bound(L, steps, max_per_cell):
    M = (4 ** L.dims) * max_per_cell
    return steps * L.dt * sum(2.0 / L.dx[a] for a in range(L.dims)) * M * 2.0 ** -41


def _continuity(dims, n, dxl, ppc, slab, steps, sigma, lib=None):
    w = S.base(name="thermal", dims=dims, n=list(n), dx_lambda=list(dxl), ppc=ppc,
               x0_lambda=slab[0], thickness_lambda=slab[1], a0=0.0, ncs=False, brem=False,
               ne_over_nc=20.0, seed=31)
    o = oracle.OracleSim(w, _tables(), nthreads=8, lib=lib)
    L = Layout(o, dims)
    x, p, tau = _thermal(o, sigma, 17)
    o.set_electrons(x, p, tau)
    e0 = o.electrons()
    o.step(steps)
    e1 = o.electrons()
    r0 = _rho_nodes(L, e0["x"], e0["w"], e0["alive"])
    r1 = _rho_nodes(L, e1["x"], e1["w"], e1["alive"])
    res = np.abs(_div_E(L, o.fields()) - (r1 - r0))
    # nodes whose divergence stencil no absorbing face and no absorbed
    # electron's deposit window reaches
    sel = L.interior(4)
    bound = current_rounding_bound(L, steps, 4 * ppc)
    o.close()
    return float(res[sel].max()), bound, float(np.abs(r0).max())


def check_continuity(lib=None):
    """Charge conservation of the deposit in 2D and 3D: with a thermal
    plasma and no laser, div E - (rho - rho_0) stays zero on every node up to
    the stated rounding bound of the fixed-point current."""
    out = []
    for args in ((2, [40, 32], [1 / 32, 1 / 24], 4, (0.3, 0.6), 40, 0.08),
                 (3, [20, 16, 14], [1 / 16, 1 / 14, 1 / 12], 2, (0.4, 0.5), 25, 0.08)):
        res, bound, rho = _continuity(*args, lib=lib)
        assert res <= bound, (args[0], res, bound, rho)
        out.append((res, bound, rho))
    return out


def test_charge_continuity_2d_3d_within_rounding_bound(oracle_lib):
    out = check_continuity()
    print(out)
    # the bound is not vacuous: it is far below the charge density itself
    for res, bound, rho in out:
        assert bound < 1e-6 * rho


def check_current_quantum(lib=None):
    """The current as stored is a multiple of 2^-40 whose units are those of
    J (the electron's charge -w/V times its velocity): a lone electron
    drifting at v across the interior of one cell (no cell face crossed)
    carries a total current sum_nodes J_a dV = -w v_a, within the rounding
    of its contributions."""
    worst = 0.0
    for dims, n, dxl in ((2, [16, 16], [1 / 16, 1 / 16]), (3, [12, 12, 12], [1 / 12, 1 / 12, 1 / 12])):
        w = S.base(name="drift", dims=dims, n=list(n), dx_lambda=list(dxl), ppc=1,
                   x0_lambda=6 * dxl[0], thickness_lambda=dxl[0], a0=0.0, ncs=False, brem=False,
                   ne_over_nc=3.0, seed=2)
        o = oracle.OracleSim(w, _tables(), nthreads=1, lib=lib)
        L = Layout(o, dims)
        e = o.electrons()
        x = e["x"].copy()
        v = np.array([0.011, -0.007, 0.004])
        for a in range(dims):
            x[:, a] = (np.floor(x[:, a] / L.dx[a]) + 0.4) * L.dx[a]
        p = np.tile(v / math.sqrt(1 - v @ v), (o.N, 1))
        o.set_electrons(x, p, e["tau"])
        o.step(1)
        J = o.current().astype(np.float64) * 2.0 ** -40
        V = float(np.prod(L.dx[:dims]))
        wt = float(e["w"][0])
        for a in range(3):
            tot = J[a].sum() * V
            want = -wt * v[a] * o.N
            nc = o.N * 54
            worst = max(worst, abs(tot - want) / (nc * 2.0 ** -41 * V + 1e-300) / 1e6)
            assert abs(tot - want) <= nc * 2.0 ** -41 * V + 1e-12 * abs(want), (dims, a, tot, want)
        o.close()
    return worst


def test_current_units_and_quantum(oracle_lib):
    check_current_quantum()


def check_jz_path_average(lib=None):
    """In 2D3V the out-of-plane current of an electron that stays inside one
    cell is v_z times its charge density averaged over the straight path of
    the step (the density on the nodes is linear in time along the path):
    compared with that average taken by brute force, 4000 points along the
    path."""
    w = S.base(name="jz", dims=2, n=[16, 16], dx_lambda=[1 / 16, 1 / 12], ppc=1,
               x0_lambda=7 / 16, thickness_lambda=1 / 16, a0=0.0, ncs=False, brem=False,
               ne_over_nc=2.0, seed=3)
    o = oracle.OracleSim(w, _tables(), nthreads=1, lib=lib)
    L = Layout(o, 2)
    e = o.electrons()
    rng = np.random.default_rng(8)
    x = e["x"].copy()
    # start in the lower-left part of its cell, move up and right within it
    for a in range(2):
        x[:, a] = (np.floor(x[:, a] / L.dx[a]) + rng.uniform(0.05, 0.4, o.N)) * L.dx[a]
    v = np.zeros((o.N, 3))
    v[:, 0] = rng.uniform(0.2, 0.5, o.N) * L.dx[0] / L.dt
    v[:, 1] = rng.uniform(0.2, 0.5, o.N) * L.dx[1] / L.dt
    v[:, 2] = rng.uniform(-0.6, 0.6, o.N)
    v *= 0.9 / np.maximum(np.linalg.norm(v, axis=1), 0.9)[:, None]
    g = 1.0 / np.sqrt(1.0 - (v ** 2).sum(1))
    o.set_electrons(x, v * g[:, None], e["tau"])
    o.step(1)
    Jz = o.current()[2].astype(np.float64) * 2.0 ** -40
    # the node density averaged along the path, times v_z
    ts = (np.arange(4000) + 0.5) / 4000
    ref = np.zeros(L.size)
    for t in ts:
        xt = x + t * v * L.dt
        ref += _rho_nodes_vz(L, xt, e["w"], v[:, 2])
    ref /= len(ts)
    err = np.abs(Jz - ref).max()
    o.close()
    assert err <= 1e-6 * np.abs(ref).max(), (err, np.abs(ref).max())
    return err


def _rho_nodes_vz(L, x, w, vz):
    return _rho_nodes(L, x, w * vz, np.ones(len(w), dtype=bool))


def test_jz_is_the_path_average_2d(oracle_lib):
    print(check_jz_path_average())


# ------------------------------------------------------ Gaussian beam
def _beam_fit(L, Ey, x_plane, kx, half_width):
    """Amplitude and phase of Ey ~ A(y) sin(kx x - phi(y)) in a window of
    +-half_width around x = x_plane, per transverse row (least squares in
    x); returns transverse coordinates, amplitude and phase arrays."""
    X = L.pos(ESTAG[1])
    sel = np.abs(X[0] - x_plane) <= half_width
    rows = {}
    for idx in np.nonzero(sel)[0]:
        key = tuple(L.ijk[1:, idx])
        rows.setdefault(key, []).append(idx)
    out = []
    for key, ids in rows.items():
        ids = np.array(ids)
        xs = X[0, ids]
        M = np.stack([np.sin(kx * xs), np.cos(kx * xs)], axis=1)
        (a, b), *_ = np.linalg.lstsq(M, Ey[ids], rcond=None)
        # a sin + b cos = A sin(kx x + d)
        out.append((X[1, ids[0]], X[2, ids[0]], math.hypot(a, b), math.atan2(b, a)))
    return np.array(out)


def _gauss_width(r, A):
    """Fit A = A0 exp(-r^2 / w^2) by least squares on ln A (rows above 5%
    of the peak)."""
    m = A > 0.05 * A.max()
    c = np.polyfit(r[m] ** 2, np.log(A[m]), 1)
    return 1.0 / math.sqrt(-c[0]), math.exp(c[1])


def _gaussian_beam(dims, lib=None):
    """Vacuum run of the laser source with a Gaussian profile; returns the
    fitted waist (in lambda), on-axis amplitude (in a0) and on-axis phase at
    the focal plane and one plane further along."""
    if dims == 2:
        w0l, dxl, n = 2.0, 1 / 32, [640, 544]
        dz = 1.0            # second plane: one Rayleigh length past focus
        xf = 4 / 32 + 0.5 * math.pi * w0l ** 2
        dur = 24.0
    else:
        w0l, dxl, n = 1.5, 1 / 12, [120, 96, 96]
        dz = 0.6            # second plane: 0.6 Rayleigh lengths past focus
        xf = 4 / 12 + 0.6 * math.pi * w0l ** 2
        dur = 20.0
    zR = math.pi * w0l ** 2
    planes = [xf, xf + dz * zR]
    w = S.base(name="beam", dims=dims, n=n, dx_lambda=[dxl] * dims, ppc=1, x0_lambda=0.0,
               thickness_lambda=0.0, a0=1.0, w0_lambda=w0l, focus_x_lambda=xf,
               duration_cycles=dur, ncs=False, brem=False)
    o = oracle.OracleSim(w, _tables(), nthreads=8, lib=lib)
    L = Layout(o, dims)
    dt = L.dt
    # on-axis numerical wave number of the Yee scheme along x: sin(k dx/2)/dx = sin(dt/2)/dt
    kx = 2.0 / L.dx[0] * math.asin(L.dx[0] / dt * math.sin(dt / 2))
    res = []
    t_done = 0
    for xp in planes:
        # envelope peak (emitted at half the pulse) reaches the plane
        t = (0.5 * dur + xp) * TWOPI
        nstep = int(round(t / dt))
        o.step(nstep - t_done)
        t_done = nstep
        fit = _beam_fit(L, o.fields()[1], xp * TWOPI, kx, 0.5 * TWOPI)
        yc = 0.5 * L.n[1] * L.dx[1]
        zc = 0.5 * L.n[2] * L.dx[2] if dims == 3 else 0.0
        if dims == 3:
            # the axis row: y at half-integers, z at integers around the centre
            r = np.hypot(fit[:, 0] - yc, fit[:, 1] - zc)
        else:
            r = np.abs(fit[:, 0] - yc)
        wz, A0 = _gauss_width(r, fit[:, 2])
        axis = np.argmin(r)
        res.append(dict(w=wz / TWOPI, A=A0, d=fit[axis, 3], t=nstep * dt))
    o.close()
    return res, w0l, zR, dz, kx


def check_gaussian_beam(dims, lib=None):
    """Paraxial Gaussian beam: waist w0 at the focal plane and w0 sqrt(1 +
    z^2) at z Rayleigh lengths past it; on-axis amplitude a0 at focus,
    falling as w0/w (3D) or sqrt(w0/w) (2D); Gouy phase atan(z) (3D) or
    atan(z)/2 (2D) gained between the two planes."""
    res, w0l, zR, dz, kx = _gaussian_beam(dims, lib)
    f, s = res
    w_exp = w0l * math.sqrt(1 + dz * dz)
    ratio = (w0l / w_exp) if dims == 3 else math.sqrt(w0l / w_exp)
    gouy = math.atan(dz) * (1.0 if dims == 3 else 0.5)
    # On axis Ey ~ A sin(t - kx (x - x_s) + psi(x)), psi the Gouy phase, zero
    # at focus (the source's phase is referred to the focal plane).  A fit of
    # sin(kx x + d) over x at time t gives psi(x) - kx x_s = pi - t - d (mod 2 pi).
    wrap = lambda a: (a + math.pi) % TWOPI - math.pi
    x_s = 4 * (TWOPI / (32 if dims == 2 else 12))
    psi_f = wrap(math.pi - f["t"] - f["d"] - kx * x_s)
    dpsi = wrap((math.pi - s["t"] - s["d"]) - (math.pi - f["t"] - f["d"]))
    rep = dict(w_focus=f["w"], w_far=s["w"], A_focus=f["A"], A_ratio=s["A"] / f["A"],
               gouy=dpsi, psi_focus=psi_f, want=dict(w0=w0l, w=w_exp, ratio=ratio, gouy=gouy))
    assert abs(f["w"] / w0l - 1) < 0.03, rep
    assert abs(s["w"] / w_exp - 1) < 0.03, rep
    assert abs(f["A"] - 1.0) < 0.04, rep
    assert abs(s["A"] / f["A"] / ratio - 1) < 0.03, rep
    assert abs(dpsi - gouy) < 0.06, rep
    assert abs(psi_f) < 0.06, rep
    return rep


@pytest.mark.slow
def test_gaussian_beam_2d_paraxial(oracle_lib):
    print(check_gaussian_beam(2))


@pytest.mark.slow
def test_gaussian_beam_3d_paraxial(oracle_lib):
    print(check_gaussian_beam(3))


# ----------------------------------------------------- absorbing faces
def check_mur_absorbs(lib=None):
    """A pulse launched by the source leaves through the first-order Mur
    faces at normal incidence: after it has gone, the box holds less than 1%
    of the pulse's peak field (1D plane wave; 2D wide Gaussian beam)."""
    out = []
    for dims, n, dxl, w0 in ((1, [512], [1 / 32], 0.0), (2, [256, 256], [1 / 32, 1 / 32], 3.0)):
        w = S.base(name="mur", dims=dims, n=n, dx_lambda=dxl, ppc=1, x0_lambda=0.0,
                   thickness_lambda=0.0, a0=1.0, w0_lambda=w0, focus_x_lambda=4.0,
                   duration_cycles=4.0, ncs=False, brem=False)
        o = oracle.OracleSim(w, _tables(), nthreads=8, lib=lib)
        dt = o.derived()["dt"]
        peak = 0.0
        # the pulse needs 4 periods to be emitted and L/c to cross the box
        total = int((4.0 + n[0] * dxl[0] + 1.0) * TWOPI / dt)
        for _ in range(8):
            o.step(total // 8)
            peak = max(peak, np.abs(o.fields()[1]).max())
        o.step(int(2.0 * TWOPI / dt))
        left = np.abs(o.fields()).max()
        o.close()
        assert left < 0.01 * peak, (dims, left, peak)
        out.append((left, peak))
    return out


def test_mur_faces_absorb(oracle_lib):
    print(check_mur_absorbs())
