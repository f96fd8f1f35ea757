"""CPU checks of the C-ABI library: it loads, exports every function that
include/nb.h declares, and its host-only entry points (version, status text,
defaults, workspace sizing, argument validation) behave.  No compute call is
made here; those need a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nb.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(nb_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def nb():
    from paper_2601_19654_amd import nb as m
    m.lib()
    return m


def test_every_declared_symbol_is_exported(nb):
    names = _declared()
    assert len(names) >= 18
    for name in names:
        assert hasattr(nb.lib(), name), name
    assert set(names) == set(nb.SIGNATURES), set(names) ^ set(nb.SIGNATURES)


def test_version_status_defaults(nb):
    assert nb.version() == (0, 3)
    assert nb.strerror(nb.NB_E_CAPACITY).startswith("encounter")
    p = nb.default_params()
    assert abs(p.G - (0.01720209895 * 365.25) ** 2) < 1e-14
    assert p.n_hill == 3.0 and p.chg_inner == 0.1 and p.mode == nb.NB_FP64
    assert abs(p.drag_sigma0 - 1.1252e-4) < 1e-7


def _wsize(nb, off, enc_cap=1024, nbig=None, **kw):
    p = nb.default_params(**kw)
    off = np.ascontiguousarray(off, dtype=np.int32)
    nb_arr = None if nbig is None else np.ascontiguousarray(nbig, dtype=np.int32)
    n = ctypes.c_size_t()
    rc = nb.lib().nb_workspace_size(ctypes.byref(p), len(off) - 1, off.ctypes.data_as(ctypes.c_void_p),
                                    None if nb_arr is None else nb_arr.ctypes.data_as(ctypes.c_void_p),
                                    enc_cap, ctypes.byref(n))
    return rc, n.value


def test_workspace_size_and_validation(nb):
    rc, a = _wsize(nb, [0, 1000])
    assert rc == 0 and a > 1000 * 17 * 8
    rc, b = _wsize(nb, [0, 4000])
    assert rc == 0 and b > a
    rc, c = _wsize(nb, [0, 400, 400, 1000])       # an empty system is allowed
    assert rc == 0
    assert _wsize(nb, [0, 10, 5])[0] == nb.NB_E_INVALID          # decreasing offsets
    assert _wsize(nb, [1, 10])[0] == nb.NB_E_INVALID             # off[0] != 0
    assert _wsize(nb, [0, 0])[0] == nb.NB_E_INVALID              # no bodies
    assert _wsize(nb, [0, 10], mode=7)[0] == nb.NB_E_INVALID
    assert _wsize(nb, [0, 10], force_r=3)[0] == nb.NB_E_INVALID
    assert _wsize(nb, [0, 10], G=-1.0)[0] == nb.NB_E_INVALID
    assert _wsize(nb, [0, 10], enc_cap=-1)[0] == nb.NB_E_INVALID
    # big/small split: 0 <= nbig[s] <= N_s; no drag with small bodies
    assert _wsize(nb, [0, 400, 1000], nbig=[400, 10])[0] == 0
    assert _wsize(nb, [0, 400, 1000], nbig=[400, 0])[0] == 0
    assert _wsize(nb, [0, 400, 1000], nbig=[401, 10])[0] == nb.NB_E_INVALID
    assert _wsize(nb, [0, 400, 1000], nbig=[-1, 10])[0] == nb.NB_E_INVALID
    assert _wsize(nb, [0, 400, 1000], nbig=[400, 10], drag=1)[0] == nb.NB_E_INVALID
    assert _wsize(nb, [0, 400, 1000], nbig=[400, 600], drag=1)[0] == 0
    # resolver parameters
    assert _wsize(nb, [0, 10], resolve=2)[0] == nb.NB_E_INVALID
    assert _wsize(nb, [0, 10], resolve=1, step_algo=2)[0] == nb.NB_E_INVALID
    assert _wsize(nb, [0, 10], resolve=1, bs_tol=-1.0)[0] == nb.NB_E_INVALID
    # the resolver's buffers grow with the list capacity (records of both ends of
    # every listed pair), beyond what the list itself takes
    plain = [_wsize(nb, [0, 1000], enc_cap=cap)[1] for cap in (1024, 2048)]
    full = [_wsize(nb, [0, 1000], enc_cap=cap, resolve=1)[1] for cap in (1024, 2048)]
    assert full[1] - full[0] > plain[1] - plain[0] > 0
    # encounter check against the big bodies only: at most 256 big bodies per system
    assert _wsize(nb, [0, 1000], nbig=[100], enc_algo=3)[0] == 0
    assert _wsize(nb, [0, 1000], enc_algo=3)[0] == nb.NB_E_INVALID
    assert _wsize(nb, [0, 1000], enc_algo=5)[0] == nb.NB_E_INVALID

def test_create_rejects_bad_workspace(nb):
    p = nb.default_params()
    off = np.array([0, 10], dtype=np.int32)
    ctx = ctypes.c_void_p()
    rc = nb.lib().nb_create(ctypes.byref(p), 1, off.ctypes.data_as(ctypes.c_void_p), None, 16, None, 0,
                            None, ctypes.byref(ctx))
    assert rc == nb.NB_E_WORKSPACE and not ctx.value
    rc = nb.lib().nb_create(ctypes.byref(p), 1, off.ctypes.data_as(ctypes.c_void_p), None, 16,
                            ctypes.c_void_p(0x1001), 1 << 20, None, ctypes.byref(ctx))
    assert rc == nb.NB_E_WORKSPACE


def test_tuning_table_read_by_the_library(nb, tmp_path):
    """nb_params.autotune_path: the library itself applies the table's entry for
    the GPU, mode and size class when the tile fields are 0 (on this host there
    is no GPU, so the class's architecture is 'unknown')."""
    off = [0, 1000]
    t = tmp_path / "tuning.tsv"
    t.write_text("# key force_algo force_r force_jchunk enc_algo enc_jchunk step_algo\n"
                 "unknown/fp64/n1024/s1 1 4 256 1 512 1\n"
                 "unknown/fp32c/n1024/s1 2 1 1024 2 1024 1\n")
    path = str(t).encode()
    rc, tuned = _wsize(nb, off, autotune_path=path)
    rc2, explicit = _wsize(nb, off, force_algo=1, force_r=4, force_jchunk=256, enc_algo=1, enc_jchunk=512,
                           step_algo=1)
    rc3, default = _wsize(nb, off)
    assert rc == rc2 == rc3 == 0
    assert tuned == explicit != default
    rc, tuned32 = _wsize(nb, off, mode=nb.NB_FP32C, autotune_path=path)
    rc2, explicit32 = _wsize(nb, off, mode=nb.NB_FP32C, force_algo=2, force_r=1, enc_algo=2)
    assert rc == rc2 == 0 and tuned32 == explicit32
    # a class the table lacks keeps the defaults; an explicit field turns the table off
    assert _wsize(nb, [0, 3000], autotune_path=path)[1] == _wsize(nb, [0, 3000])[1]
    assert _wsize(nb, off, force_r=2, autotune_path=path)[1] == _wsize(nb, off, force_r=2)[1]
    # an unreadable table is an error
    assert _wsize(nb, off, autotune_path=str(tmp_path / "missing.tsv").encode())[0] == nb.NB_E_INVALID


def test_package_tuning_table_matches_the_autotuner_cache():
    from paper_2601_19654_amd import autotune
    cache = autotune.load_cache()
    rows = {}
    for line in open(autotune.TABLE):
        if line.startswith("#"):
            continue
        k, *vals = line.split()
        rows[k] = [int(v) for v in vals]
    assert set(rows) == set(cache)
    for k, vals in rows.items():
        assert vals == [int(cache[k].get(f, 0)) for f in autotune.TABLE_FIELDS], k


def test_workspace_stays_bounded_for_millions_of_bodies(nb):
    """The symmetric force's split partials grow as N^2/T; beyond 4 GiB of them
    the automatic choice takes ordered pairs with at most 64 source chunks, so
    the workspace grows about linearly: 2^21 bodies in one system fit in a few
    GiB of the 288 GB of HBM (the sorted encounter check's tile-pair list is
    the largest part there)."""
    p = nb.default_params()
    sizes = {}
    for n in (131072, 600000, 1 << 21):
        off = np.array([0, n], np.int32)
        b = ctypes.c_size_t()
        assert nb.lib().nb_workspace_size(ctypes.byref(p), 1, off.ctypes.data_as(ctypes.c_void_p), None,
                                          1 << 18, ctypes.byref(b)) == nb.NB_OK
        sizes[n] = b.value
    assert sizes[600000] < 4 << 30
    assert sizes[1 << 21] < 16 << 30

