"""Shared fixtures.  GPU tests are marked ``gpu``; everything else runs on CPU."""
from __future__ import annotations

import hashlib
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: longer CPU test")


def _cache_dir():
    d = os.path.join(ROOT, "_build", "cache")
    os.makedirs(d, exist_ok=True)
    return d


def oracle_tables(Z: int, k_cut: float = 1.0) -> dict:
    """Oracle-built emission tables (cached on disk, keyed by the builder's
    source text)."""
    from oracle import tables as T
    src = open(os.path.join(ROOT, "oracle", "tables.py"), "rb").read()
    key = hashlib.sha256(src + f"{Z}:{k_cut!r}".encode()).hexdigest()[:16]
    path = os.path.join(_cache_dir(), f"oracle_tables_{Z}_{key}.npz")
    if os.path.exists(path):
        d = dict(np.load(path))
    else:
        d = T.build_tables(Z, k_cut)
        tmp = path + f".{os.getpid()}.tmp.npz"
        np.savez(tmp, **d)
        os.replace(tmp, path)
        d = dict(np.load(path))
    for k in ("n_eta", "n_xi", "n_T", "n_y", "Z"):
        d[k] = int(d[k])
    for k in ("ln_eta0", "dln_eta", "ln_T0", "dln_T", "k_cut"):
        d[k] = float(d[k])
    return d


@pytest.fixture(scope="session")
def tables_al():
    return oracle_tables(13)


@pytest.fixture(scope="session")
def tables_au():
    return oracle_tables(79)


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    oracle.build(force=False)
    return oracle


@pytest.fixture(scope="session")
def gpu_lib():
    """The HIP library; GPU tests fail (not skip) when it cannot run."""
    from paper_1612_07592_amd import binding
    L = binding.load()
    return binding
