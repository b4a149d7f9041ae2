"""FP64 CPU oracle for the per-electron PIC step with MC photon emission.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import, build or run anything here; the
product path (the HIP library and its Python binding) never does.  The oracle
shares no code with the HIP library: it has its own Philox, its own field
solver, pusher, emission modules and its own table quadrature
(``oracle/tables.py``).  The only inputs both sides see are the workload
recipes (``paper_1612_07592_amd/workloads.py``, data only) and, in parity
tests, the same table arrays.

Build: ``build()`` compiles ``oracle.c`` with gcc, ``-O2 -ffp-contract=off``
(no FMA contraction, no fast-math, sin and cos kept as separate libm calls)
and OpenMP.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")

OR_NCS, OR_BREM, OR_FROZEN, OR_NO_RECOIL, OR_BREM_FREEPATH = 1, 2, 4, 16, 32
OR_BW, OR_BH = 64, 128
FROZEN_UNIFORM, FROZEN_PLANE_WAVE = 0, 1


def _stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(os.path.join(HERE, f)) > t for f in ("oracle.c", "oracle.h"))


def build(force: bool = True) -> str:
    """Compile the oracle shared library in place (always when force, else
    only when it is missing or older than its sources); returns its path."""
    if not force and not _stale():
        return LIB
    tmp = LIB + ".tmp"
    compile_source(os.path.join(HERE, "oracle.c"), tmp)
    os.replace(tmp, LIB)
    return LIB


def compile_source(src: str, out: str) -> str:
    """gcc of one oracle source file (oracle.h beside it) into a shared
    object, with the oracle's flags."""
    # -fno-builtin-sin/-cos: keep sin and cos separate libm calls (gcc would
    # otherwise merge them into sincos, whose results can differ by an ulp)
    cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off", "-fno-fast-math",
           "-fno-builtin-sin", "-fno-builtin-cos", "-fopenmp", "-fPIC", "-shared", src, "-o", out,
           "-lm"]
    subprocess.run(cmd, check=True)
    return out


class _Cfg(C.Structure):
    _fields_ = [("dims", C.c_int32), ("flags", C.c_int32), ("frozen_kind", C.c_int32),
                ("ppc", C.c_int32), ("n", C.c_int32 * 3), ("Z", C.c_int32),
                ("charge_state", C.c_int32), ("dx_lambda", C.c_double * 3),
                ("cfl", C.c_double), ("lambda_m", C.c_double), ("a0", C.c_double),
                ("w0_lambda", C.c_double), ("duration_cycles", C.c_double),
                ("focus_x_lambda", C.c_double), ("ne_over_nc", C.c_double),
                ("x0_lambda", C.c_double), ("thickness_lambda", C.c_double),
                ("photon_cut_mc2", C.c_double), ("frozen_E", C.c_double * 3),
                ("frozen_B", C.c_double * 3), ("frozen_a", C.c_double),
                ("seed", C.c_uint64), ("job_id", C.c_uint64), ("photon_capacity", C.c_uint64),
                ("ion_ppc", C.c_int32), ("envelope", C.c_int32), ("ion_mass", C.c_double),
                ("pair_capacity", C.c_uint64)]


class _Tab(C.Structure):
    _fields_ = [("n_eta", C.c_int32), ("n_xi", C.c_int32), ("ln_eta0", C.c_double),
                ("dln_eta", C.c_double), ("h", C.POINTER(C.c_double)),
                ("ln_xi", C.POINTER(C.c_double)), ("ncs_cdf", C.POINTER(C.c_double)),
                ("n_T", C.c_int32), ("n_y", C.c_int32), ("ln_T0", C.c_double),
                ("dln_T", C.c_double), ("k_cut", C.c_double),
                ("sigma", C.POINTER(C.c_double)), ("br_cdf", C.POINTER(C.c_double)),
                ("n_chi", C.c_int32), ("n_xp", C.c_int32), ("ln_chi0", C.c_double),
                ("dln_chi", C.c_double), ("bw_lnT", C.POINTER(C.c_double)),
                ("bw_cdf", C.POINTER(C.c_double)), ("n_k", C.c_int32), ("n_s", C.c_int32),
                ("ln_k0", C.c_double), ("dln_k", C.c_double),
                ("bh_sigma", C.POINTER(C.c_double)), ("bh_cdf", C.POINTER(C.c_double))]


class _Stats(C.Structure):
    _fields_ = [("steps", C.c_uint64), ("live", C.c_uint64), ("events", C.c_uint64 * 2),
                ("kept", C.c_uint64 * 2), ("dropped_ncs", C.c_uint64),
                ("overflow", C.c_uint64), ("brem_clamped", C.c_uint64),
                ("e_rad_kept", C.c_double * 2), ("e_rad_dropped", C.c_double),
                ("ions_live", C.c_uint64), ("pairs", C.c_uint64 * 2),
                ("pairs_overflow", C.c_uint64), ("e_pair", C.c_double * 2),
                ("spectrum", (C.c_uint64 * 64) * 2)]


_libs = {}


def _load(path=None):
    """The oracle library (built in place when stale), or the shared object
    at `path` built from a copy of the same sources (the pins' planted-error
    checks compile altered copies)."""
    key = path or LIB
    if key not in _libs:
        if path is None and _stale():
            build()
        L = C.CDLL(key)
        P = C.c_void_p
        L.or_create.restype = P
        L.or_create.argtypes = [C.POINTER(_Cfg), C.POINTER(_Tab), C.c_int]
        L.or_destroy.argtypes = [P]
        L.or_step.argtypes = [P, C.c_int]
        L.or_num_electrons.restype = C.c_int64
        L.or_num_electrons.argtypes = [P]
        L.or_num_photons.restype = C.c_int64
        L.or_num_photons.argtypes = [P]
        L.or_get_electrons.argtypes = [P] + [C.c_void_p] * 6
        L.or_set_electrons.argtypes = [P] + [C.c_void_p] * 3
        L.or_get_tau_brem.argtypes = [P, C.c_void_p]
        L.or_set_tau_brem.argtypes = [P, C.c_void_p]
        L.or_get_photons.argtypes = [P] + [C.c_void_p] * 7
        L.or_num_pairs.restype = C.c_int64
        L.or_num_pairs.argtypes = [P]
        L.or_get_pairs.argtypes = [P] + [C.c_void_p] * 9
        L.or_add_photons.argtypes = [P, C.c_int64] + [C.c_void_p] * 5
        L.or_get_flight.argtypes = [P] + [C.c_void_p] * 3
        L.or_get_stats.argtypes = [P, C.POINTER(_Stats)]
        L.or_kinetic_energy.restype = C.c_double
        L.or_kinetic_energy.argtypes = [P]
        L.or_field_energy.restype = C.c_double
        L.or_field_energy.argtypes = [P]
        L.or_field_size.restype = C.c_int64
        L.or_field_size.argtypes = [P]
        L.or_get_fields.argtypes = [P, C.c_void_p]
        L.or_get_derived.argtypes = [P, C.c_void_p]
        L.or_get_current.argtypes = [P, C.c_void_p]
        L.or_philox.argtypes = [C.c_uint32] * 6 + [C.c_void_p]
        L.or_set_fields.argtypes = [P, C.c_void_p]
        L.or_num_ions.restype = C.c_int64
        L.or_num_ions.argtypes = [P]
        L.or_get_ions.argtypes = [P, C.c_void_p, C.c_void_p, C.c_void_p]
        L.or_set_ions.argtypes = [P, C.c_void_p, C.c_void_p]
        L.or_ion_kinetic_energy.restype = C.c_double
        L.or_ion_kinetic_energy.argtypes = [P]
        L.or_math.restype = C.c_double
        L.or_math.argtypes = [C.c_int, C.c_double]
        L.or_probe_field.restype = C.c_double
        L.or_probe_field.argtypes = [P, C.c_int, C.c_void_p]
        L.or_probe_boris.argtypes = [P, C.c_void_p, C.c_void_p, C.c_void_p]
        L.or_probe_eta.restype = C.c_double
        L.or_probe_eta.argtypes = [P, C.c_void_p, C.c_void_p, C.c_void_p]
        for name in ("or_probe_ncs_dtau", "or_probe_ncs_xi", "or_probe_brem_sigma"):
            getattr(L, name).restype = C.c_double
            getattr(L, name).argtypes = [P, C.c_double, C.c_double]
        L.or_probe_brem_sigma.argtypes = [P, C.c_double]
        L.or_probe_brem_eps.restype = C.c_double
        L.or_probe_brem_eps.argtypes = [P, C.c_double, C.c_double]
        _libs[key] = L
    return _libs[key]


def philox(ctr, key):
    """Philox4x32-10 of one counter (4 words) and key (2 words)."""
    out = np.zeros(4, dtype=np.uint32)
    _load().or_philox(*[int(c) & 0xFFFFFFFF for c in ctr], *[int(k) & 0xFFFFFFFF for k in key],
                      out.ctypes.data)
    return out


def math(which: str, x, lib=None):
    """The oracle's own exp, log or expm1 (elementwise)."""
    f = _load(lib).or_math
    k = {"exp": 0, "log": 1, "expm1": 2}[which]
    return np.array([f(k, float(v)) for v in np.atleast_1d(x)])


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def flags_from(w):
    f = 0
    if w.get("ncs", True):
        f |= OR_NCS
    if w.get("brem", True):
        f |= OR_BREM
    if w.get("frozen", False):
        f |= OR_FROZEN
    if w.get("no_recoil", False):
        f |= OR_NO_RECOIL
    if w.get("brem_freepath", False):
        f |= OR_BREM_FREEPATH
    if w.get("bw", False):
        f |= OR_BW
    if w.get("bh", False):
        f |= OR_BH
    return f


class OracleSim:
    """One oracle run of a workload dict (see ``workloads.py``) and tables."""

    def __init__(self, w: dict, tables: dict, nthreads: int | None = None, lib: str | None = None):
        L = _load(lib)
        c = _Cfg()
        c.dims = int(w["dims"])
        c.flags = flags_from(w)
        c.frozen_kind = int(w.get("frozen_kind", FROZEN_UNIFORM))
        c.ppc = int(w["ppc"])
        n = list(w["n"]) + [1] * (3 - len(w["n"]))
        dx = list(w["dx_lambda"]) + [1.0] * (3 - len(w["dx_lambda"]))
        for a in range(3):
            c.n[a] = int(n[a])
            c.dx_lambda[a] = float(dx[a])
        c.Z = int(w["Z"])
        c.charge_state = int(w["charge_state"])
        c.cfl = float(w.get("cfl", 0.95))
        c.lambda_m = float(w.get("lambda_m", 1e-6))
        c.a0 = float(w.get("a0", 0.0))
        c.w0_lambda = float(w.get("w0_lambda", 0.0))
        c.duration_cycles = float(w.get("duration_cycles", 10.0))
        c.focus_x_lambda = float(w.get("focus_x_lambda", 0.0))
        c.ne_over_nc = float(w["ne_over_nc"])
        c.x0_lambda = float(w["x0_lambda"])
        c.thickness_lambda = float(w["thickness_lambda"])
        c.photon_cut_mc2 = float(w.get("photon_cut_mc2", 1.0))
        fe = list(w.get("frozen_E", [0.0, 0.0, 0.0]))
        fb = list(w.get("frozen_B", [0.0, 0.0, 0.0]))
        for a in range(3):
            c.frozen_E[a] = float(fe[a])
            c.frozen_B[a] = float(fb[a])
        c.frozen_a = float(w.get("frozen_a", 0.0))
        c.seed = int(w.get("seed", 1))
        c.job_id = int(w.get("job_id", 0))
        c.photon_capacity = int(w.get("photon_capacity", 1 << 20))
        c.ion_ppc = int(w.get("ion_ppc", 0))
        c.envelope = 1 if w.get("envelope", "sin2") == "flat" else 0
        c.ion_mass = float(w.get("ion_mass_me", 0.0))
        c.pair_capacity = int(w.get("pair_capacity", 1 << 16))
        self._keep = []
        t = _Tab()
        t.n_eta = int(tables["n_eta"]); t.n_xi = int(tables["n_xi"])
        t.ln_eta0 = float(tables["ln_eta0"]); t.dln_eta = float(tables["dln_eta"])
        t.n_T = int(tables["n_T"]); t.n_y = int(tables["n_y"])
        t.ln_T0 = float(tables["ln_T0"]); t.dln_T = float(tables["dln_T"])
        t.k_cut = float(tables["k_cut"])
        for name in ("h", "ln_xi", "ncs_cdf", "sigma", "br_cdf"):
            a = np.ascontiguousarray(tables[name], dtype=np.float64)
            self._keep.append(a)
            setattr(t, name, _dptr(a))
        if "bw_lnT" in tables:
            t.n_chi = int(tables["n_chi"]); t.n_xp = int(tables["n_xp"])
            t.ln_chi0 = float(tables["ln_chi0"]); t.dln_chi = float(tables["dln_chi"])
            t.n_k = int(tables["n_k"]); t.n_s = int(tables["n_s"])
            t.ln_k0 = float(tables["ln_k0"]); t.dln_k = float(tables["dln_k"])
            for name in ("bw_lnT", "bw_cdf", "bh_sigma", "bh_cdf"):
                a = np.ascontiguousarray(tables[name], dtype=np.float64)
                self._keep.append(a)
                setattr(t, name, _dptr(a))
        elif flags_from(w) & (OR_BW | OR_BH):
            raise ValueError("pair production needs the pair tables (oracle.tables.build_bw/build_bh)")
        nt = nthreads if nthreads is not None else min(os.cpu_count() or 1, 16)
        self._h = L.or_create(C.byref(c), C.byref(t), int(nt))
        self._L = L
        self.nthreads = nt
        self.N = int(L.or_num_electrons(self._h))
        self.Ni = int(L.or_num_ions(self._h))
        self.workload = dict(w)

    def close(self):
        if getattr(self, "_h", None):
            self._L.or_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n: int = 1):
        self._L.or_step(self._h, int(n))

    def electrons(self):
        N = self.N
        x = np.zeros((N, 3)); p = np.zeros((N, 3)); tau = np.zeros(N); w = np.zeros(N)
        i = np.zeros(N, dtype=np.uint32); al = np.zeros(N, dtype=np.uint8)
        self._L.or_get_electrons(self._h, x.ctypes.data, p.ctypes.data, tau.ctypes.data,
                                 w.ctypes.data, i.ctypes.data, al.ctypes.data)
        return dict(x=x, p=p, tau=tau, w=w, id=i, alive=al.astype(bool))

    def set_electrons(self, x, p, tau):
        x = np.ascontiguousarray(x, dtype=np.float64).reshape(self.N, 3)
        p = np.ascontiguousarray(p, dtype=np.float64).reshape(self.N, 3)
        tau = np.ascontiguousarray(tau, dtype=np.float64).reshape(self.N)
        self._L.or_set_electrons(self._h, x.ctypes.data, p.ctypes.data, tau.ctypes.data)

    def ions(self):
        """Mobile ions in id order: x, p (per unit mass), alive."""
        n = self.Ni
        x = np.zeros((n, 3)); p = np.zeros((n, 3)); al = np.zeros(n, dtype=np.uint8)
        if n:
            self._L.or_get_ions(self._h, x.ctypes.data, p.ctypes.data, al.ctypes.data)
        return dict(x=x, p=p, alive=al.astype(bool))

    def set_ions(self, x, p):
        x = np.ascontiguousarray(x, dtype=np.float64).reshape(self.Ni, 3)
        p = np.ascontiguousarray(p, dtype=np.float64).reshape(self.Ni, 3)
        self._L.or_set_ions(self._h, x.ctypes.data, p.ctypes.data)

    def ion_kinetic_energy(self):
        return float(self._L.or_ion_kinetic_energy(self._h))

    def tau_brem(self):
        """Collision optical depths of the free-path form, id order."""
        out = np.zeros(self.N)
        self._L.or_get_tau_brem(self._h, out.ctypes.data)
        return out

    def set_tau_brem(self, t):
        t = np.ascontiguousarray(t, dtype=np.float64).reshape(self.N)
        self._L.or_set_tau_brem(self._h, t.ctypes.data)

    def photons(self):
        n_all = int(self._L.or_num_photons(self._h))
        n = min(n_all, int(self.workload.get("photon_capacity", 1 << 20)))
        x = np.zeros((n, 3)); k = np.zeros((n, 3)); e = np.zeros(n); w = np.zeros(n)
        st = np.zeros(n, dtype=np.uint32); par = np.zeros(n, dtype=np.uint32)
        pr = np.zeros(n, dtype=np.uint32)
        if n:
            self._L.or_get_photons(self._h, x.ctypes.data, k.ctypes.data, e.ctypes.data,
                                   w.ctypes.data, st.ctypes.data, par.ctypes.data, pr.ctypes.data)
        return dict(x=x, k=k, energy=e, w=w, step=st, parent=par, proc=pr)

    def pairs(self):
        n_all = int(self._L.or_num_pairs(self._h))
        n = min(n_all, int(self.workload.get("pair_capacity", 1 << 16)))
        x = np.zeros((n, 3)); k = np.zeros((n, 3)); em = np.zeros(n); ep = np.zeros(n)
        w = np.zeros(n)
        st, par, pst, pr = (np.zeros(n, dtype=np.uint32) for _ in range(4))
        if n:
            self._L.or_get_pairs(self._h, x.ctypes.data, k.ctypes.data, em.ctypes.data,
                                 ep.ctypes.data, w.ctypes.data, st.ctypes.data, par.ctypes.data,
                                 pst.ctypes.data, pr.ctypes.data)
        return dict(x=x, k=k, e_minus=em, e_plus=ep, w=w, step=st, parent=par, pstep=pst,
                    proc=pr)

    def add_photons(self, x, k, eps, w, parent):
        """Append photons as records of the coming step (test hook)."""
        x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 3)
        n = x.shape[0]
        k = np.ascontiguousarray(k, dtype=np.float64).reshape(n, 3)
        eps = np.ascontiguousarray(eps, dtype=np.float64).reshape(n)
        w = np.ascontiguousarray(w, dtype=np.float64).reshape(n)
        parent = np.ascontiguousarray(parent, dtype=np.uint32).reshape(n)
        self._L.or_add_photons(self._h, n, x.ctypes.data, k.ctypes.data, eps.ctypes.data,
                               w.ctypes.data, parent.ctypes.data)

    def flight(self):
        """Photons in flight: position, pair optical depth, state."""
        n = min(int(self._L.or_num_photons(self._h)), int(self.workload.get("photon_capacity", 1 << 20)))
        x = np.zeros((n, 3)); tau = np.zeros(n); st = np.zeros(n, dtype=np.uint8)
        if n:
            self._L.or_get_flight(self._h, x.ctypes.data, tau.ctypes.data, st.ctypes.data)
        return dict(x=x, tau=tau, state=st)

    def stats(self):
        s = _Stats()
        self._L.or_get_stats(self._h, C.byref(s))
        return dict(steps=s.steps, live=s.live, events=[s.events[0], s.events[1]],
                    kept=[s.kept[0], s.kept[1]], dropped_ncs=s.dropped_ncs,
                    overflow=s.overflow, brem_clamped=s.brem_clamped,
                    e_rad_kept=[s.e_rad_kept[0], s.e_rad_kept[1]],
                    e_rad_dropped=s.e_rad_dropped, ions_live=s.ions_live,
                    pairs=[s.pairs[0], s.pairs[1]], pairs_overflow=s.pairs_overflow,
                    e_pair=[s.e_pair[0], s.e_pair[1]],
                    spectrum=np.array([list(s.spectrum[0]), list(s.spectrum[1])], dtype=np.uint64))

    def kinetic_energy(self):
        return float(self._L.or_kinetic_energy(self._h))

    def field_energy(self):
        return float(self._L.or_field_energy(self._h))

    def fields(self):
        m = int(self._L.or_field_size(self._h))
        out = np.zeros(6 * m)
        self._L.or_get_fields(self._h, out.ctypes.data)
        return out.reshape(6, m)

    def current(self):
        m = int(self._L.or_field_size(self._h))
        out = np.zeros(3 * m, dtype=np.int64)
        self._L.or_get_current(self._h, out.ctypes.data)
        return out.reshape(3, m)

    def set_fields(self, F):
        """Overwrite E and B (shape (6, size), the layout of fields())."""
        m = int(self._L.or_field_size(self._h))
        F = np.ascontiguousarray(F, dtype=np.float64).reshape(6 * m)
        self._L.or_set_fields(self._h, F.ctypes.data)

    # --- probes of single steps of the method (pins) ----------------------
    def probe_field(self, comp, x):
        """Gathered component comp (0..2 E, 3..5 B) at position x[3]."""
        x = np.ascontiguousarray(x, dtype=np.float64).reshape(3)
        return float(self._L.or_probe_field(self._h, int(comp), x.ctypes.data))

    def probe_boris(self, E, B, p):
        E = np.ascontiguousarray(E, dtype=np.float64).reshape(3)
        B = np.ascontiguousarray(B, dtype=np.float64).reshape(3)
        q = np.array(p, dtype=np.float64).reshape(3)
        self._L.or_probe_boris(self._h, E.ctypes.data, B.ctypes.data, q.ctypes.data)
        return q

    def probe_eta(self, E, B, p):
        E = np.ascontiguousarray(E, dtype=np.float64).reshape(3)
        B = np.ascontiguousarray(B, dtype=np.float64).reshape(3)
        p = np.ascontiguousarray(p, dtype=np.float64).reshape(3)
        return float(self._L.or_probe_eta(self._h, E.ctypes.data, B.ctypes.data, p.ctypes.data))

    def probe_ncs_dtau(self, eta, gamma):
        return float(self._L.or_probe_ncs_dtau(self._h, float(eta), float(gamma)))

    def probe_ncs_xi(self, eta, u):
        u = np.atleast_1d(np.asarray(u, dtype=np.float64))
        f = self._L.or_probe_ncs_xi
        return np.array([f(self._h, float(eta), float(v)) for v in u])

    def probe_brem_sigma(self, T):
        return float(self._L.or_probe_brem_sigma(self._h, float(T)))

    def probe_brem_eps(self, T, u):
        u = np.atleast_1d(np.asarray(u, dtype=np.float64))
        f = self._L.or_probe_brem_eps
        return np.array([f(self._h, float(T), float(v)) for v in u])

    def derived(self):
        o = np.zeros(8)
        self._L.or_get_derived(self._h, o.ctypes.data)
        return dict(dx=o[0:3].copy(), dt=o[3], E_S=o[4], K_N=o[5], K_BR=o[6], n_c=o[7])
