"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point declared in include/dbm.h, and rejects invalid
configurations before touching the device."""
import ctypes
import os
import re

import pytest

from paper_2006_15932_amd import dbm as D
from paper_2006_15932_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "dbm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dbm_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 12
    L = D.lib()
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(D.SIGNATURES)


def _cfg(p, **kw):
    return D.Configs([p.with_(**kw)] if kw else [p])


def test_workspace_bytes_is_positive_and_scales():
    p = W.reacting(n=64, steps=1)
    b64 = D.dbm_workspace_bytes(D.Configs([p], "fp64"))
    b32 = D.dbm_workspace_bytes(D.Configs([p], "fp32"))
    assert b64 > 0 and b32 > 0 and b32 < b64
    # three f buffers at least
    assert b32 >= 3 * 3 * 16 * 64 * 64 * 4
    # four times the cells: about four times the bytes (each plane of the f
    # buffers also carries a fixed pad of a few KiB)
    mid = D.dbm_workspace_bytes(D.Configs([W.reacting(n=256, steps=1)], "fp32"))
    big = D.dbm_workspace_bytes(D.Configs([W.reacting(n=512, steps=1)], "fp32"))
    assert 3.8 < big / mid < 4.2
    assert big >= 3 * 3 * 16 * 512 * 512 * 4


@pytest.mark.parametrize("bad,code", [
    (dict(nx=0), D.DBM_ERR_ARG),
    (dict(ny=-3), D.DBM_ERR_ARG),
    (dict(dt=0.0), D.DBM_ERR_ARG),
    (dict(dx=float("nan")), D.DBM_ERR_ARG),
    (dict(bc_x=7), D.DBM_ERR_ARG),
    (dict(scheme=5), D.DBM_ERR_ARG),
])
def test_create_rejects_bad_grid(bad, code):
    p = W.reacting(n=16, steps=1)
    cfg = D.Configs([p.with_(**bad)])
    assert D.dbm_workspace_bytes(cfg) == 0
    with pytest.raises(D.DbmError) as e:
        D.dbm_create(cfg, 0, 0, 0)
    assert e.value.code == code


def test_create_rejects_bad_species_and_reaction():
    p = W.reacting(n=16, steps=1)
    sp = list(p.species)
    sp[1] = W.Species(m=-2.0)
    with pytest.raises(D.DbmError) as e:
        D.dbm_create(D.Configs([p.with_(species=sp)]), 0, 0, 0)
    assert e.value.code == D.DBM_ERR_ARG
    sp = [W.make_species(2.0, tau=1e-5, a=-2), W.make_species(32.0, tau=3e-5, a=-1),
          W.make_species(18.0, a=2)]
    with pytest.raises(D.DbmError) as e:
        D.dbm_create(D.Configs([p.with_(species=sp)]), 0, 0, 0)
    assert e.value.code == D.DBM_ERR_UNSUPPORTED
    with pytest.raises(D.DbmError) as e:
        D.dbm_create(D.Configs([p.with_(reaction=dict(fuel=0, oxid=0, k_ov=1.0, Ea_over_R=1.0))]),
                     0, 0, 0)
    assert e.value.code == D.DBM_ERR_ARG


def test_create_rejects_singular_moment_matrix():
    p = W.reacting(n=16, steps=1)
    sp = [W.Species(m=1.0, eta=(0.5, 0.5, 0.5, 0.5))] * 3
    with pytest.raises(D.DbmError) as e:
        D.dbm_create(D.Configs([p.with_(species=sp, reaction=None)]), 0, 0, 0)
    assert e.value.code == D.DBM_ERR_SINGULAR_M
    assert "singular" in D.last_error()


def test_create_rejects_missing_or_small_workspace():
    p = W.reacting(n=16, steps=1)
    cfg = D.Configs([p])
    with pytest.raises(D.DbmError) as e:
        D.dbm_create(cfg, 0, 0, 1 << 30)
    assert e.value.code == D.DBM_ERR_WORKSPACE
    with pytest.raises(D.DbmError) as e:
        D.dbm_create(cfg, 0, 4096, 16)
    assert e.value.code == D.DBM_ERR_WORKSPACE


def test_batch_must_share_template_parameters():
    a = W.reacting(n=16, steps=1)
    b = W.reacting(n=32, steps=1).with_(scheme=W.RK3)
    cfg = D.Configs([a, b])
    assert D.dbm_workspace_bytes(cfg) == 0
    with pytest.raises(D.DbmError) as e:
        D.dbm_create(cfg, 0, 0, 0)
    assert e.value.code == D.DBM_ERR_UNSUPPORTED


def test_null_handle_calls_fail_cleanly():
    L = D.lib()
    assert L.dbm_step(None, 1) == D.DBM_ERR_ARG
    assert L.dbm_destroy(None) == D.DBM_ERR_ARG
    assert L.dbm_moments(None, 0, None, None, None, None) == D.DBM_ERR_ARG
    assert L.dbm_state_bytes(None, 0) == 0
    assert L.dbm_save_state(None, 0, None, 0) == D.DBM_ERR_ARG
    assert L.dbm_load_state(None, 0, None, 0) == D.DBM_ERR_ARG


@pytest.mark.parametrize("src,dst,nbytes,grid,reps", [
    (0, 1 << 20, 4096, 64, 1),            # null source
    (1 << 20, 0, 4096, 64, 1),            # null destination
    (1 << 20, 1 << 24, 4100, 64, 1),      # not a multiple of 16 bytes
    (1 << 20, 1 << 24, 0, 64, 1),         # empty
    (1 << 20, (1 << 20) + 8, 4096, 64, 1),  # misaligned and overlapping
    (1 << 20, (1 << 20) + 1024, 4096, 64, 1),  # overlapping
    (1 << 20, 1 << 24, 4096, 0, 1),       # no workgroups
    (1 << 20, 1 << 24, 4096, 64, 0),      # no repetitions
])
def test_copy_rate_rejects_bad_arguments_before_any_launch(src, dst, nbytes, grid, reps):
    # the addresses are never dereferenced: validation happens on the host
    with pytest.raises(D.DbmError) as e:
        D.dbm_copy_rate(src, dst, nbytes, grid, reps, 0)
    assert e.value.code == D.DBM_ERR_ARG


@pytest.mark.parametrize("words", [0, 3, 5, 16])
def test_copy_rate_rejects_unsupported_words_in_flight(words):
    with pytest.raises(D.DbmError) as e:
        D.dbm_copy_rate(1 << 20, 1 << 24, 4096, 64, 1, 0, words)
    assert e.value.code == D.DBM_ERR_ARG


def test_binding_constants_match_the_header():
    """Every DBM_* enumerator the binding names has the header's value."""
    import re
    hdr = open(os.path.join(ROOT, "include", "dbm.h")).read()
    body = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    vals = {}
    for blk in re.findall(r"enum\s*\{(.*?)\}", body, flags=re.S):
        for name, v in re.findall(r"(DBM_\w+)\s*=\s*(-?\d+)", blk):
            vals[name] = int(v)
    seen = 0
    for name in dir(D):
        if name.startswith("DBM_") and name in vals:
            assert getattr(D, name) == vals[name], name
            seen += 1
    assert seen >= 20
    assert D.DBM_OPT_ROUNDING == vals["DBM_OPT_ROUNDING"] == 10


def test_plain_c_consumer_builds_links_and_runs(tmp_path):
    """The header compiles as strict C99 and the library links and runs
    from C (host-only entry points; no GPU)."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    lib_dir = os.path.dirname(D.LIB_PATH)
    exe = str(tmp_path / "abi_consumer")
    cmd = [cc, "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror",
           "-I", os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "abi_consumer.c"),
           "-o", exe, "-L", lib_dir, "-ldbm", "-Wl,-rpath," + lib_dir]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0 and r.stdout.startswith("OK"), (r.stdout, r.stderr)
