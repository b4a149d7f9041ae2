"""ctypes binding of libpic (include/pic.h): the same entry points by name,
argument marshalling only.  Every step of the method runs in the HIP kernels of
libpic.so; there is no Python or CPU fallback, and loading fails loudly when
the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpic.so")

PIC_ABI_VERSION = 2
PIC_TABLES_VERSION = 2
PIC_FP64, PIC_FP32_MIXED = 0, 1
PIC_NCS, PIC_BREM, PIC_FIELDS_FROZEN, PIC_NO_RECOIL, PIC_BREM_FREEPATH = 1, 2, 4, 16, 32
PIC_BW, PIC_BH = 64, 128
PIC_PAIR_TABLES_VERSION = 1
PIC_FROZEN_UNIFORM, PIC_FROZEN_PLANE_WAVE = 0, 1
PIC_ENV_SIN2, PIC_ENV_FLAT = 0, 1
STATUS = {0: "PIC_OK", 1: "PIC_ERR_INVALID", 2: "PIC_ERR_NOMEM", 3: "PIC_ERR_DEVICE",
          4: "PIC_ERR_STATE", 5: "PIC_ERR_OVERFLOW", 6: "PIC_ERR_TABLES"}

EXPORTS = ["pic_create", "pic_load_tables", "pic_step", "pic_emission_stats", "pic_destroy",
           "pic_last_error", "pic_memory_required", "pic_counts", "pic_copy_electrons",
           "pic_set_electrons", "pic_copy_photons", "pic_field_size", "pic_copy_fields",
           "pic_build_tables", "pic_philox", "pic_derived", "pic_profile", "pic_profile_read",
           "pic_copy_current", "pic_batch_create", "pic_batch_destroy", "pic_batch_last_error",
           "pic_step_many", "pic_server_create", "pic_server_destroy", "pic_server_clock",
           "pic_server_last_error", "pic_server_submit", "pic_server_run", "pic_server_poll",
           "pic_server_job_ctx", "pic_server_release", "pic_device_memory", "pic_synchronize",
           "pic_copy_brem_depth", "pic_set_brem_depth", "pic_get_buffers", "pic_philox_noalloc",
           "pic_ion_count", "pic_copy_ions", "pic_set_ions", "pic_build_pair_tables",
           "pic_load_pair_tables", "pic_pair_counts", "pic_copy_pairs", "pic_copy_flight",
           "pic_add_photons"]


class pic_config(C.Structure):
    _fields_ = [("abi_version", C.c_uint32), ("dims", C.c_uint32), ("precision", C.c_uint32),
                ("flags", C.c_uint32), ("n", C.c_int32 * 3), ("ppc", C.c_int32),
                ("Z", C.c_uint32), ("charge_state", C.c_uint32), ("frozen_kind", C.c_uint32),
                ("dx_lambda", C.c_double * 3), ("cfl", C.c_double), ("lambda_m", C.c_double),
                ("a0", C.c_double), ("w0_lambda", C.c_double), ("duration_cycles", C.c_double),
                ("focus_x_lambda", C.c_double), ("ne_over_nc", C.c_double),
                ("x0_lambda", C.c_double), ("thickness_lambda", C.c_double),
                ("photon_cut_mc2", C.c_double), ("frozen_E", C.c_double * 3),
                ("frozen_B", C.c_double * 3), ("frozen_a", C.c_double),
                ("photon_capacity", C.c_uint64), ("seed", C.c_uint64), ("job_id", C.c_uint64),
                ("sort_every", C.c_int32), ("ion_ppc", C.c_int32), ("ion_mass_me", C.c_double), ("pair_capacity", C.c_uint64),
                ("envelope", C.c_uint32), ("reserved0", C.c_uint32), ("stream", C.c_void_p)]


class pic_tables(C.Structure):
    _fields_ = [("version", C.c_uint32), ("Z", C.c_uint32), ("k_cut_mc2", C.c_double),
                ("n_eta", C.c_int32), ("n_xi", C.c_int32), ("ln_eta0", C.c_double),
                ("dln_eta", C.c_double), ("h", C.POINTER(C.c_double)),
                ("ln_xi", C.POINTER(C.c_double)), ("ncs_cdf", C.POINTER(C.c_double)),
                ("n_T", C.c_int32), ("n_y", C.c_int32), ("ln_T0", C.c_double),
                ("dln_T", C.c_double), ("sigma", C.POINTER(C.c_double)),
                ("br_cdf", C.POINTER(C.c_double)), ("checksum", C.c_uint64)]


class pic_stats(C.Structure):
    _fields_ = [("steps", C.c_uint64), ("electrons_live", C.c_uint64),
                ("electron_steps", C.c_uint64), ("events", C.c_uint64 * 2),
                ("kept", C.c_uint64 * 2), ("dropped_ncs", C.c_uint64), ("overflow", C.c_uint64),
                ("brem_clamped", C.c_uint64), ("photons_stored", C.c_uint64),
                ("untiled_steps", C.c_uint64),
                ("e_rad_kept", C.c_double * 2), ("e_rad_dropped", C.c_double),
                ("e_kin_e", C.c_double), ("e_field", C.c_double),
                ("ions_live", C.c_uint64), ("e_kin_i", C.c_double),
                ("pairs", C.c_uint64 * 2), ("pairs_stored", C.c_uint64),
                ("pairs_overflow", C.c_uint64), ("e_pair", C.c_double * 2),
                ("spectrum", (C.c_uint64 * 64) * 2)]


class pic_pair_tables(C.Structure):
    _fields_ = [("version", C.c_uint32), ("Z", C.c_uint32), ("n_chi", C.c_int32),
                ("n_xp", C.c_int32), ("ln_chi0", C.c_double), ("dln_chi", C.c_double),
                ("bw_lnT", C.POINTER(C.c_double)), ("bw_cdf", C.POINTER(C.c_double)),
                ("n_k", C.c_int32), ("n_s", C.c_int32), ("ln_k0", C.c_double),
                ("dln_k", C.c_double), ("bh_sigma", C.POINTER(C.c_double)),
                ("bh_cdf", C.POINTER(C.c_double)), ("checksum", C.c_uint64)]


class pic_server_config(C.Structure):
    _fields_ = [("abi_version", C.c_uint32), ("max_jobs", C.c_int32),
                ("quantum_steps", C.c_int32), ("keep_finished", C.c_uint32),
                ("hbm_reserve_bytes", C.c_uint64), ("stream", C.c_void_p)]


class pic_job_result(C.Structure):
    _fields_ = [("job", C.c_uint64), ("status", C.c_int32), ("steps", C.c_int32),
                ("t_submit", C.c_double), ("t_admit", C.c_double), ("t_finish", C.c_double),
                ("device_bytes", C.c_uint64), ("stats", pic_stats)]


class PicError(RuntimeError):
    def __init__(self, fn, code, msg):
        super().__init__(f"{fn} -> {STATUS.get(code, code)}: {msg}")
        self.code = code


_lib = None


def load() -> C.CDLL:
    """Load libpic.so (built by ``paper_1612_07592_amd.build``); no fallback."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libpic.so not built ({LIB_PATH}); run python -m paper_1612_07592_amd.build")
    src = os.path.join(HERE, "csrc")
    newest = max(os.path.getmtime(os.path.join(src, f)) for f in os.listdir(src))
    if newest > os.path.getmtime(LIB_PATH) + 1.0:
        import warnings
        warnings.warn("libpic.so is older than its sources; rebuild with "
                      "python -m paper_1612_07592_amd.build", RuntimeWarning)
    L = C.CDLL(LIB_PATH)
    P = C.c_void_p
    i32, u32, u64, dbl = C.c_int32, C.c_uint32, C.c_uint64, C.c_double
    L.pic_create.argtypes = [C.POINTER(pic_config), C.POINTER(P)]
    L.pic_load_tables.argtypes = [P, C.POINTER(pic_tables)]
    L.pic_step.argtypes = [P, i32]
    L.pic_emission_stats.argtypes = [P, C.POINTER(pic_stats)]
    L.pic_destroy.argtypes = [P]
    L.pic_destroy.restype = None
    L.pic_last_error.argtypes = [P]
    L.pic_last_error.restype = C.c_char_p
    L.pic_memory_required.argtypes = [C.POINTER(pic_config), C.POINTER(u64)]
    L.pic_counts.argtypes = [P, C.POINTER(u64), C.POINTER(u64), C.POINTER(u64)]
    L.pic_copy_electrons.argtypes = [P] + [C.c_void_p] * 6
    L.pic_set_electrons.argtypes = [P] + [C.c_void_p] * 3
    L.pic_copy_brem_depth.argtypes = [P, C.c_void_p]
    L.pic_get_buffers.argtypes = [P, C.c_void_p]
    L.pic_set_brem_depth.argtypes = [P, C.c_void_p]
    L.pic_copy_photons.argtypes = [P, u64, u64] + [C.c_void_p] * 7
    L.pic_field_size.argtypes = [P, C.POINTER(u64)]
    L.pic_copy_fields.argtypes = [P, C.c_void_p]
    L.pic_build_tables.argtypes = [u32, dbl, i32] + [C.c_void_p] * 5 + [C.POINTER(pic_tables)]
    L.pic_philox.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, u64]
    L.pic_philox_noalloc.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, u64]
    L.pic_derived.argtypes = [P, C.c_void_p]
    L.pic_ion_count.argtypes = [P, C.POINTER(u64)]
    L.pic_build_pair_tables.argtypes = [u32, i32] + [C.c_void_p] * 4 + [C.POINTER(pic_pair_tables)]
    L.pic_load_pair_tables.argtypes = [P, C.POINTER(pic_pair_tables)]
    L.pic_pair_counts.argtypes = [P, C.POINTER(u64), C.POINTER(u64)]
    L.pic_copy_pairs.argtypes = [P, u64, u64] + [C.c_void_p] * 9
    L.pic_copy_flight.argtypes = [P, u64, u64] + [C.c_void_p] * 3
    L.pic_add_photons.argtypes = [P, u64] + [C.c_void_p] * 5
    L.pic_copy_ions.argtypes = [P, C.c_void_p, C.c_void_p, C.c_void_p]
    L.pic_set_ions.argtypes = [P, C.c_void_p, C.c_void_p]
    L.pic_copy_current.argtypes = [P, C.c_void_p]
    L.pic_profile.argtypes = [P, i32]
    L.pic_profile_read.argtypes = [P, C.c_void_p, C.c_void_p]
    L.pic_batch_create.argtypes = [P, C.POINTER(P)]
    L.pic_batch_destroy.argtypes = [P]
    L.pic_batch_destroy.restype = None
    L.pic_batch_last_error.argtypes = [P]
    L.pic_batch_last_error.restype = C.c_char_p
    L.pic_step_many.argtypes = [P, C.c_void_p, C.c_void_p, i32]
    L.pic_server_create.argtypes = [C.POINTER(pic_server_config), C.POINTER(P)]
    L.pic_server_destroy.argtypes = [P]
    L.pic_server_destroy.restype = None
    L.pic_server_clock.argtypes = [P]
    L.pic_server_clock.restype = C.c_double
    L.pic_server_last_error.argtypes = [P]
    L.pic_server_last_error.restype = C.c_char_p
    L.pic_server_submit.argtypes = [P, C.POINTER(pic_config), C.POINTER(pic_tables), i32, dbl,
                                    C.POINTER(u64)]
    L.pic_server_run.argtypes = [P, C.POINTER(i32), C.POINTER(i32)]
    L.pic_server_poll.argtypes = [P, C.c_void_p, i32, C.POINTER(i32)]
    L.pic_server_job_ctx.argtypes = [P, u64, C.POINTER(P)]
    L.pic_server_release.argtypes = [P, u64]
    L.pic_device_memory.argtypes = [C.POINTER(u64), C.POINTER(u64)]
    L.pic_synchronize.argtypes = [P]
    no_status = ("pic_destroy", "pic_last_error", "pic_batch_destroy", "pic_batch_last_error",
                 "pic_server_destroy", "pic_server_clock", "pic_server_last_error")
    for name in EXPORTS:
        fn = getattr(L, name)
        if name not in no_status:
            fn.restype = C.c_int
    _lib = L
    return L


def _check(fn, code, ctx=None, ok=(0,)):
    if code not in ok:
        msg = load().pic_last_error(ctx)
        raise PicError(fn, code, msg.decode() if msg else "")
    return code


def config_from(w: dict, stream=None) -> pic_config:
    """pic_config from a workload recipe dict (``workloads.py`` keys)."""
    c = pic_config()
    c.abi_version = PIC_ABI_VERSION
    c.dims = int(w["dims"])
    c.precision = PIC_FP32_MIXED if w.get("precision", "fp64") == "fp32" else PIC_FP64
    f = 0
    f |= PIC_NCS if w.get("ncs", True) else 0
    f |= PIC_BREM if w.get("brem", True) else 0
    f |= PIC_FIELDS_FROZEN if w.get("frozen", False) else 0
    f |= PIC_NO_RECOIL if w.get("no_recoil", False) else 0
    f |= PIC_BREM_FREEPATH if w.get("brem_freepath", False) else 0
    f |= PIC_BW if w.get("bw", False) else 0
    f |= PIC_BH if w.get("bh", False) else 0
    c.flags = f
    n = list(w["n"]) + [1] * (3 - len(w["n"]))
    dx = list(w["dx_lambda"]) + [1.0] * (3 - len(w["dx_lambda"]))
    for a in range(3):
        c.n[a] = int(n[a])
        c.dx_lambda[a] = float(dx[a])
    c.ppc = int(w["ppc"])
    c.Z = int(w["Z"])
    c.charge_state = int(w["charge_state"])
    c.frozen_kind = int(w.get("frozen_kind", PIC_FROZEN_UNIFORM))
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
    fe = list(w.get("frozen_E", [0.0] * 3))
    fb = list(w.get("frozen_B", [0.0] * 3))
    for a in range(3):
        c.frozen_E[a] = float(fe[a])
        c.frozen_B[a] = float(fb[a])
    c.frozen_a = float(w.get("frozen_a", 0.0))
    c.photon_capacity = int(w.get("photon_capacity", 1 << 20))
    c.seed = int(w.get("seed", 1))
    c.job_id = int(w.get("job_id", 0))
    c.sort_every = int(w.get("sort_every", 0))
    c.ion_ppc = int(w.get("ion_ppc", 0))
    c.ion_mass_me = float(w.get("ion_mass_me", 0.0))
    c.pair_capacity = int(w.get("pair_capacity", 1 << 16))
    c.envelope = PIC_ENV_FLAT if w.get("envelope", "sin2") == "flat" else PIC_ENV_SIN2
    c.stream = stream
    return c


def tables_struct(t: dict):
    """pic_tables pointing at the arrays of a table dict; returns (struct, keepalive)."""
    s = pic_tables()
    s.version = PIC_TABLES_VERSION
    s.Z = int(t["Z"])
    s.k_cut_mc2 = float(t["k_cut"])
    s.n_eta, s.n_xi = int(t["n_eta"]), int(t["n_xi"])
    s.ln_eta0, s.dln_eta = float(t["ln_eta0"]), float(t["dln_eta"])
    s.n_T, s.n_y = int(t["n_T"]), int(t["n_y"])
    s.ln_T0, s.dln_T = float(t["ln_T0"]), float(t["dln_T"])
    keep = []
    for name in ("h", "ln_xi", "ncs_cdf", "sigma", "br_cdf"):
        a = np.ascontiguousarray(t[name], dtype=np.float64)
        keep.append(a)
        setattr(s, name, a.ctypes.data_as(C.POINTER(C.c_double)))
    s.checksum = int(t.get("checksum", 0))
    return s, keep


def pair_tables_struct(t: dict):
    """pic_pair_tables pointing at the pair arrays of a table dict; (struct, keepalive)."""
    s = pic_pair_tables()
    s.version = PIC_PAIR_TABLES_VERSION
    s.Z = int(t["Z"])
    s.n_chi, s.n_xp = int(t["n_chi"]), int(t["n_xp"])
    s.ln_chi0, s.dln_chi = float(t["ln_chi0"]), float(t["dln_chi"])
    s.n_k, s.n_s = int(t["n_k"]), int(t["n_s"])
    s.ln_k0, s.dln_k = float(t["ln_k0"]), float(t["dln_k"])
    keep = []
    for name in ("bw_lnT", "bw_cdf", "bh_sigma", "bh_cdf"):
        a = np.ascontiguousarray(t[name], dtype=np.float64)
        keep.append(a)
        setattr(s, name, a.ctypes.data_as(C.POINTER(C.c_double)))
    s.checksum = int(t.get("pair_checksum", 0))
    return s, keep


def pic_build_pair_tables(Z: int, nthreads: int = 0) -> dict:
    """The library's own pair-production tables as a dict of numpy arrays
    (merge into the emission-table dict for runs with PIC_BW / PIC_BH)."""
    L = load()
    bwT = np.zeros(128); bwC = np.zeros(128 * 128); bhS = np.zeros(128); bhC = np.zeros(128 * 64)
    out = pic_pair_tables()
    _check("pic_build_pair_tables", L.pic_build_pair_tables(int(Z), int(nthreads), bwT.ctypes.data,
                                                            bwC.ctypes.data, bhS.ctypes.data,
                                                            bhC.ctypes.data, C.byref(out)))
    return dict(Z=int(Z), n_chi=out.n_chi, n_xp=out.n_xp, ln_chi0=out.ln_chi0, dln_chi=out.dln_chi,
                bw_lnT=bwT, bw_cdf=bwC.reshape(128, 128), n_k=out.n_k, n_s=out.n_s,
                ln_k0=out.ln_k0, dln_k=out.dln_k, bh_sigma=bhS, bh_cdf=bhC.reshape(128, 64),
                pair_checksum=int(out.checksum))


def pic_build_tables(Z: int, k_cut_mc2: float = 1.0, nthreads: int = 0) -> dict:
    """The library's own emission tables as a dict of numpy arrays."""
    L = load()
    h = np.zeros(256); lx = np.zeros(256); ncs = np.zeros(256 * 256)
    sig = np.zeros(128); br = np.zeros(128 * 64)
    out = pic_tables()
    _check("pic_build_tables", L.pic_build_tables(int(Z), float(k_cut_mc2), int(nthreads),
                                                  h.ctypes.data, lx.ctypes.data, ncs.ctypes.data,
                                                  sig.ctypes.data, br.ctypes.data, C.byref(out)))
    return dict(Z=int(Z), k_cut=float(k_cut_mc2), n_eta=out.n_eta, n_xi=out.n_xi,
                ln_eta0=out.ln_eta0, dln_eta=out.dln_eta, h=h, ln_xi=lx,
                ncs_cdf=ncs.reshape(256, 256), n_T=out.n_T, n_y=out.n_y, ln_T0=out.ln_T0,
                dln_T=out.dln_T, sigma=sig, br_cdf=br.reshape(128, 64), checksum=int(out.checksum))


def pic_philox(ctr, key) -> np.ndarray:
    """Device Philox4x32-10 of counters ctr[n,4] under key[2]."""
    L = load()
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    key = np.ascontiguousarray(key, dtype=np.uint32).reshape(2)
    out = np.zeros_like(ctr)
    _check("pic_philox", L.pic_philox(ctr.ctypes.data, key.ctypes.data, out.ctypes.data, ctr.shape[0]))
    return out


def pic_philox_noalloc(ctr, key) -> np.ndarray:
    """pic_philox through the library's fixed device staging (no device
    allocation); at most 65536 counters per call."""
    L = load()
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    key = np.ascontiguousarray(key, dtype=np.uint32).reshape(2)
    out = np.zeros_like(ctr)
    _check("pic_philox_noalloc", L.pic_philox_noalloc(ctr.ctypes.data, key.ctypes.data, out.ctypes.data,
                                                      ctr.shape[0]))
    return out


def pic_memory_required(w: dict) -> int:
    L = load()
    c = config_from(w)
    b = C.c_uint64(0)
    _check("pic_memory_required", L.pic_memory_required(C.byref(c), C.byref(b)))
    return int(b.value)


def stats_dict(s: pic_stats, code: int = 0) -> dict:
    return dict(steps=s.steps, live=s.electrons_live, electron_steps=s.electron_steps,
                events=[s.events[0], s.events[1]], kept=[s.kept[0], s.kept[1]],
                dropped_ncs=s.dropped_ncs, overflow=s.overflow,
                brem_clamped=s.brem_clamped, photons_stored=s.photons_stored,
                untiled_steps=s.untiled_steps,
                e_rad_kept=[s.e_rad_kept[0], s.e_rad_kept[1]],
                e_rad_dropped=s.e_rad_dropped, e_kin_e=s.e_kin_e, e_field=s.e_field,
                ions_live=s.ions_live, e_kin_i=s.e_kin_i, pairs=[s.pairs[0], s.pairs[1]],
                pairs_stored=s.pairs_stored, pairs_overflow=s.pairs_overflow,
                e_pair=[s.e_pair[0], s.e_pair[1]],
                spectrum=np.array([list(s.spectrum[0]), list(s.spectrum[1])], dtype=np.uint64),
                status=STATUS.get(code, code))


def pic_device_memory():
    """(free, total) bytes of the current device, as admission sees them."""
    L = load()
    f, t = C.c_uint64(), C.c_uint64()
    _check("pic_device_memory", L.pic_device_memory(C.byref(f), C.byref(t)))
    return int(f.value), int(t.value)


class pic_buffers(C.Structure):
    """Borrowed device pointers of a context (pic_get_buffers)."""
    _fields_ = [("precision", C.c_uint32), ("dims", C.c_uint32), ("fb", C.c_int32 * 3),
                ("electrons", C.c_uint64), ("photons_stored", C.c_uint64),
                ("field_size", C.c_uint64), ("x", C.c_void_p * 3), ("p", C.c_void_p * 3),
                ("tau", C.c_void_p), ("taub", C.c_void_p), ("w", C.c_void_p), ("id", C.c_void_p),
                ("E", C.c_void_p * 3), ("B", C.c_void_p * 3), ("J", C.c_void_p * 3),
                ("photon_x", C.c_void_p * 3), ("photon_k", C.c_void_p * 3),
                ("photon_eps", C.c_void_p), ("photon_w", C.c_void_p),
                ("photon_step", C.c_void_p), ("photon_parent", C.c_void_p),
                ("photon_proc", C.c_void_p)]


class Sim:
    """One libpic context: pic_create / pic_load_tables / pic_step /
    pic_emission_stats / pic_destroy plus the copy helpers."""

    def __init__(self, w: dict, tables: dict | None = None, stream=None, _handle=None):
        L = load()
        self._L = L
        self.workload = dict(w)
        self._owned = _handle is None
        if _handle is None:
            cfg = config_from(w, stream)
            h = C.c_void_p()
            _check("pic_create", L.pic_create(C.byref(cfg), C.byref(h)))
            self._h = h
        else:
            self._h = _handle
        n = C.c_uint64()
        _check("pic_counts", L.pic_counts(self._h, C.byref(n), None, None), self._h)
        self.N = int(n.value)
        ni = C.c_uint64()
        _check("pic_ion_count", L.pic_ion_count(self._h, C.byref(ni)), self._h)
        self.Ni = int(ni.value)
        if tables is not None:
            self.pic_load_tables(tables)

    # --- the five calls ---------------------------------------------------
    def pic_load_tables(self, tables: dict):
        """Emission tables; with PIC_BW / PIC_BH also the pair tables of the
        same dict (pic_load_pair_tables)."""
        s, keep = tables_struct(tables)
        _check("pic_load_tables", self._L.pic_load_tables(self._h, C.byref(s)), self._h)
        if (self.workload.get("bw") or self.workload.get("bh")) and "bw_lnT" in tables:
            self.pic_load_pair_tables(tables)

    def pic_load_pair_tables(self, tables: dict):
        s, keep = pair_tables_struct(tables)
        _check("pic_load_pair_tables", self._L.pic_load_pair_tables(self._h, C.byref(s)), self._h)

    def pair_counts(self):
        st, cr = C.c_uint64(), C.c_uint64()
        _check("pic_pair_counts", self._L.pic_pair_counts(self._h, C.byref(st), C.byref(cr)), self._h)
        return int(st.value), int(cr.value)

    def pairs(self) -> dict:
        """Pair records (device append order)."""
        n, _ = self.pair_counts()
        x = np.zeros((n, 3)); k = np.zeros((n, 3)); em = np.zeros(n); ep = np.zeros(n)
        w = np.zeros(n)
        st, par, pst, pr = (np.zeros(n, dtype=np.uint32) for _ in range(4))
        if n:
            _check("pic_copy_pairs", self._L.pic_copy_pairs(
                self._h, 0, n, x.ctypes.data, k.ctypes.data, em.ctypes.data, ep.ctypes.data,
                w.ctypes.data, st.ctypes.data, par.ctypes.data, pst.ctypes.data, pr.ctypes.data),
                self._h)
        return dict(x=x, k=k, e_minus=em, e_plus=ep, w=w, step=st, parent=par, pstep=pst, proc=pr)

    def flight(self) -> dict:
        """State in flight of the stored photon records (record order)."""
        _, n, _ = self.counts()
        x = np.zeros((n, 3)); tau = np.zeros(n); state = np.zeros(n, dtype=np.uint8)
        if n:
            _check("pic_copy_flight", self._L.pic_copy_flight(self._h, 0, n, x.ctypes.data,
                                                              tau.ctypes.data, state.ctypes.data),
                   self._h)
        return dict(x=x, tau=tau, state=state)

    def add_photons(self, x, k, eps, w, parent):
        """Append photon records of the coming step (test hook)."""
        x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 3)
        n = x.shape[0]
        k = np.ascontiguousarray(k, dtype=np.float64).reshape(n, 3)
        eps = np.ascontiguousarray(eps, dtype=np.float64).reshape(n)
        w = np.ascontiguousarray(w, dtype=np.float64).reshape(n)
        parent = np.ascontiguousarray(parent, dtype=np.uint32).reshape(n)
        _check("pic_add_photons", self._L.pic_add_photons(self._h, n, x.ctypes.data, k.ctypes.data,
                                                          eps.ctypes.data, w.ctypes.data,
                                                          parent.ctypes.data), self._h)

    def pic_step(self, n: int = 1):
        _check("pic_step", self._L.pic_step(self._h, int(n)), self._h)

    def pic_emission_stats(self) -> dict:
        s = pic_stats()
        code = self._L.pic_emission_stats(self._h, C.byref(s))
        _check("pic_emission_stats", code, self._h, ok=(0, 5))
        return stats_dict(s, code)

    def synchronize(self):
        """Wait for this context's stream (pic_synchronize)."""
        _check("pic_synchronize", self._L.pic_synchronize(self._h), self._h)

    def pic_destroy(self):
        if getattr(self, "_h", None):
            if getattr(self, "_owned", True):
                self._L.pic_destroy(self._h)
            self._h = None

    close = pic_destroy

    def __del__(self):
        try:
            self.pic_destroy()
        except Exception:
            pass

    # --- helpers ----------------------------------------------------------
    step = pic_step
    stats = pic_emission_stats

    def counts(self):
        e, s, k = C.c_uint64(), C.c_uint64(), C.c_uint64()
        _check("pic_counts", self._L.pic_counts(self._h, C.byref(e), C.byref(s), C.byref(k)), self._h)
        return int(e.value), int(s.value), int(k.value)

    def electrons(self) -> dict:
        N = self.N
        x = np.zeros((N, 3)); p = np.zeros((N, 3)); tau = np.zeros(N); w = np.zeros(N)
        i = np.zeros(N, dtype=np.uint32); al = np.zeros(N, dtype=np.uint8)
        _check("pic_copy_electrons",
               self._L.pic_copy_electrons(self._h, x.ctypes.data, p.ctypes.data, tau.ctypes.data,
                                          w.ctypes.data, i.ctypes.data, al.ctypes.data), self._h)
        return dict(x=x, p=p, tau=tau, w=w, id=i, alive=al.astype(bool))

    def set_electrons(self, x, p, tau):
        x = np.ascontiguousarray(x, dtype=np.float64).reshape(self.N, 3)
        p = np.ascontiguousarray(p, dtype=np.float64).reshape(self.N, 3)
        tau = np.ascontiguousarray(tau, dtype=np.float64).reshape(self.N)
        _check("pic_set_electrons", self._L.pic_set_electrons(self._h, x.ctypes.data, p.ctypes.data,
                                                              tau.ctypes.data), self._h)

    def ions(self) -> dict:
        """Mobile ions in id order: x[n,3], p[n,3] (per unit mass), alive[n]."""
        n = self.Ni
        x = np.zeros((n, 3)); p = np.zeros((n, 3)); al = np.zeros(n, dtype=np.uint8)
        _check("pic_copy_ions", self._L.pic_copy_ions(self._h, x.ctypes.data, p.ctypes.data,
                                                      al.ctypes.data), self._h)
        return dict(x=x, p=p, alive=al.astype(bool))

    def set_ions(self, x, p):
        x = np.ascontiguousarray(x, dtype=np.float64).reshape(self.Ni, 3)
        p = np.ascontiguousarray(p, dtype=np.float64).reshape(self.Ni, 3)
        _check("pic_set_ions", self._L.pic_set_ions(self._h, x.ctypes.data, p.ctypes.data), self._h)

    def buffers(self) -> dict:
        """Borrowed device pointers (ints) and sizes, valid until the next step."""
        b = pic_buffers()
        _check("pic_get_buffers", self._L.pic_get_buffers(self._h, C.byref(b)), self._h)
        out = {}
        for name, _ in pic_buffers._fields_:
            v = getattr(b, name)
            out[name] = list(v) if isinstance(v, C.Array) else v
        return out

    def brem_depth(self) -> np.ndarray:
        """Collision optical depths of a free-path bremsstrahlung run, id order."""
        out = np.zeros(self.N)
        _check("pic_copy_brem_depth", self._L.pic_copy_brem_depth(self._h, out.ctypes.data), self._h)
        return out

    def set_brem_depth(self, t):
        t = np.ascontiguousarray(t, dtype=np.float64).reshape(self.N)
        _check("pic_set_brem_depth", self._L.pic_set_brem_depth(self._h, t.ctypes.data), self._h)

    def photons(self, off: int = 0, n: int | None = None) -> dict:
        _, stored, _ = self.counts()
        if n is None:
            n = stored - off
        x = np.zeros((n, 3)); k = np.zeros((n, 3)); e = np.zeros(n); w = np.zeros(n)
        st = np.zeros(n, dtype=np.uint32); par = np.zeros(n, dtype=np.uint32)
        pr = np.zeros(n, dtype=np.uint32)
        _check("pic_copy_photons",
               self._L.pic_copy_photons(self._h, int(off), int(n), x.ctypes.data, k.ctypes.data,
                                        e.ctypes.data, w.ctypes.data, st.ctypes.data,
                                        par.ctypes.data, pr.ctypes.data), self._h)
        return dict(x=x, k=k, energy=e, w=w, step=st, parent=par, proc=pr)

    def fields(self) -> np.ndarray:
        m = C.c_uint64()
        _check("pic_field_size", self._L.pic_field_size(self._h, C.byref(m)), self._h)
        out = np.zeros(6 * int(m.value))
        _check("pic_copy_fields", self._L.pic_copy_fields(self._h, out.ctypes.data), self._h)
        return out.reshape(6, int(m.value))

    def profile(self, enable: bool = True):
        _check("pic_profile", self._L.pic_profile(self._h, 1 if enable else 0), self._h)

    def profile_read(self):
        """ms and launch counts: [electron step, field solve, sort, ions, photons]."""
        ms = np.zeros(5)
        n = np.zeros(5, dtype=np.uint64)
        _check("pic_profile_read", self._L.pic_profile_read(self._h, ms.ctypes.data, n.ctypes.data), self._h)
        return ms, n

    def current(self) -> np.ndarray:
        """J^{n+1/2} of the last step, int64 in units of 2^-40, shape (3, size)."""
        m = C.c_uint64()
        _check("pic_field_size", self._L.pic_field_size(self._h, C.byref(m)), self._h)
        out = np.zeros(3 * int(m.value), dtype=np.int64)
        _check("pic_copy_current", self._L.pic_copy_current(self._h, out.ctypes.data), self._h)
        return out.reshape(3, int(m.value))

    def derived(self) -> dict:
        o = np.zeros(8)
        _check("pic_derived", self._L.pic_derived(self._h, o.ctypes.data), self._h)
        return dict(dx=o[0:3].copy(), dt=o[3], E_S=o[4], K_N=o[5], K_BR=o[6], n_c=o[7])


class Batch:
    """pic_batch_create / pic_step_many / pic_batch_destroy: several runs
    advanced with one launch per kernel and step."""

    def __init__(self, stream=None):
        self._L = load()
        h = C.c_void_p()
        code = self._L.pic_batch_create(stream, C.byref(h))
        if code:
            raise PicError("pic_batch_create", code, "")
        self._h = h

    def step_many(self, sims, nsteps):
        n = len(sims)
        ctxs = (C.c_void_p * max(n, 1))(*[s._h for s in sims])
        steps = (C.c_int32 * max(n, 1))(*[int(k) for k in nsteps])
        code = self._L.pic_step_many(self._h, ctxs, steps, n)
        if code:
            raise PicError("pic_step_many", code, self._L.pic_batch_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            self._L.pic_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """The continuous-batching scan-job server of libpic (pic_server_*)."""

    def __init__(self, max_jobs=64, quantum_steps=16, keep_finished=False,
                 hbm_reserve_bytes=8 << 30, stream=None):
        self._L = load()
        sc = pic_server_config()
        sc.abi_version = PIC_ABI_VERSION
        sc.max_jobs = int(max_jobs)
        sc.quantum_steps = int(quantum_steps)
        sc.keep_finished = 1 if keep_finished else 0
        sc.hbm_reserve_bytes = int(hbm_reserve_bytes)
        sc.stream = stream
        h = C.c_void_p()
        code = self._L.pic_server_create(C.byref(sc), C.byref(h))
        if code:
            raise PicError("pic_server_create", code, "")
        self._h = h
        self._keep = []

    def _err(self, fn, code):
        raise PicError(fn, code, self._L.pic_server_last_error(self._h).decode())

    def clock(self) -> float:
        return float(self._L.pic_server_clock(self._h))

    def submit(self, w: dict, tables: dict | None, nsteps: int, t_arrival: float = -1.0) -> int:
        cfg = config_from(w)
        job = C.c_uint64()
        if tables is not None:
            ts, keep = tables_struct(tables)
            code = self._L.pic_server_submit(self._h, C.byref(cfg), C.byref(ts), int(nsteps),
                                             float(t_arrival), C.byref(job))
        else:
            code = self._L.pic_server_submit(self._h, C.byref(cfg), None, int(nsteps),
                                             float(t_arrival), C.byref(job))
        if code:
            self._err("pic_server_submit", code)
        return int(job.value)

    def run(self):
        """One scheduling round; returns (resident, queued)."""
        r, q = C.c_int32(), C.c_int32()
        code = self._L.pic_server_run(self._h, C.byref(r), C.byref(q))
        if code:
            self._err("pic_server_run", code)
        return int(r.value), int(q.value)

    def poll(self, max_results: int = 1024) -> list:
        out = (pic_job_result * max_results)()
        n = C.c_int32()
        code = self._L.pic_server_poll(self._h, out, int(max_results), C.byref(n))
        if code:
            self._err("pic_server_poll", code)
        res = []
        for k in range(n.value):
            r = out[k]
            res.append(dict(job=int(r.job), status=STATUS.get(r.status, r.status), steps=int(r.steps),
                            t_submit=r.t_submit, t_admit=r.t_admit, t_finish=r.t_finish,
                            device_bytes=int(r.device_bytes), stats=stats_dict(r.stats)))
        return res

    def job_sim(self, job: int, w: dict) -> Sim:
        """Borrowed view of a finished job's context (keep_finished servers)."""
        h = C.c_void_p()
        code = self._L.pic_server_job_ctx(self._h, int(job), C.byref(h))
        if code:
            self._err("pic_server_job_ctx", code)
        return Sim(w, None, _handle=h)

    def release(self, job: int):
        code = self._L.pic_server_release(self._h, int(job))
        if code:
            self._err("pic_server_release", code)

    def close(self):
        if getattr(self, "_h", None):
            self._L.pic_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
