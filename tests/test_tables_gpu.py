"""pic_load_tables rejects bad tables with PIC_ERR_TABLES and leaves the
context usable; stepping before any tables is PIC_ERR_STATE."""
from __future__ import annotations

import numpy as np
import pytest

import scenarios as S

pytestmark = pytest.mark.gpu


def _bad(t, **kw):
    u = {k: (np.array(v, copy=True) if isinstance(v, np.ndarray) else v) for k, v in t.items()}
    u.update(kw)
    return u


def test_bad_tables_rejected_and_context_survives(gpu_lib):
    print("\n[gpu-case] PIC_ERR_TABLES rejections", flush=True)
    good = gpu_lib.pic_build_tables(13, 1.0, 16)
    w = S.c1_parity(16)
    g = gpu_lib.Sim(w, None)
    with pytest.raises(gpu_lib.PicError) as e:
        g.pic_step(1)
    assert e.value.code == 4                      # PIC_ERR_STATE: emission on, no tables
    cases = {}
    cases["Z"] = _bad(good, Z=79)
    h = good["h"].copy(); h[17] = np.nan
    cases["nan h"] = _bad(good, h=h)
    c = good["ncs_cdf"].copy(); c[40, 100], c[40, 101] = c[40, 101], c[40, 100] - 1e-3
    cases["ncs row not monotone"] = _bad(good, ncs_cdf=c)
    b = good["br_cdf"].copy(); b[90, -1] = 0.999
    cases["brem row end"] = _bad(good, br_cdf=b)
    s = good["sigma"].copy(); s[100] *= 1.0 + 1e-12      # a row above the photon cut (sigma > 0)
    assert s[100] != good["sigma"][100]
    cases["checksum"] = _bad(good, sigma=s)       # altered after it was built
    lx = good["ln_xi"].copy(); lx[10] = lx[9]
    cases["ln_xi not increasing"] = _bad(good, ln_xi=lx)
    accepted = []
    for name, t in cases.items():
        try:
            g.pic_load_tables(t)
            accepted.append(name)
        except gpu_lib.PicError as e:
            assert e.code == 6, (name, e)           # PIC_ERR_TABLES
    assert not accepted, accepted
    import ctypes as C
    ts, keep = gpu_lib.tables_struct(good)
    ts.version = 1
    assert gpu_lib.load().pic_load_tables(g._h, C.byref(ts)) == 6   # wrong layout version
    # the same altered sigma without a checksum passes every other check
    g.pic_load_tables(_bad(good, sigma=s, checksum=0))
    g.pic_load_tables(good)
    g.pic_step(16)
    st = g.stats()
    assert st["steps"] == 16 and st["live"] == g.N
    g.close()
