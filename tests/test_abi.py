"""The C-ABI library loads and exports every entry point that include/mdlbm.h
declares; host-only argument checks work without a GPU."""
import ctypes
import re
from pathlib import Path

import pytest

from paper_2206_11634_amd import binding as B

ROOT = Path(__file__).resolve().parents[1]
HEADER = ROOT / "include" / "mdlbm.h"


def _declared():
    text = HEADER.read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\**\s+\**(\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    if not B.LIB_PATH.exists():
        from paper_2206_11634_amd import build
        build.build()
    return B.load()


def test_header_declares_the_hot_path_calls():
    names = _declared()
    for n in ("lbm_init", "lbm_classify_nodes", "lbm_step", "lbm_particle_forces", "dem_step"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
    assert set(B.EXPORTS) == set(names)


def _cfg(**kw):
    c = B.LbmConfig()
    c.nx, c.ny, c.nz = kw.get("dims", (16, 12, 10))
    c.periodic = (ctypes.c_int32 * 3)(*kw.get("periodic", (1, 0, 1)))
    c.tau = kw.get("tau", 0.8)
    c.rho0 = 1.0
    c.storage = kw.get("storage", 1)
    c.treatments = 3
    c.n_particles = kw.get("n_particles", 0)
    c.box_half = kw.get("box_half", 4)
    return c


@pytest.mark.parametrize("storage,es", [(0, 8), (1, 4), (2, 2)])
def test_query_sizes(lib, storage, es):
    s = B.lbm_query_sizes(_cfg(storage=storage))
    assert s.ncell == 16 * 12 * 10
    assert s.cell_stride % 64 == 0 and s.cell_stride >= s.ncell
    assert s.population_bytes == 19 * s.cell_stride * es
    assert s.owner_bytes == 4 * s.ncell and s.flag_bytes == s.ncell
    assert s.moment_bytes == 4 * es * s.ncell


def test_init_rejects_unknown_classify_mode(lib):
    bufs = B.LbmBuffers()
    ctx = ctypes.c_void_p()
    cfg = _cfg()
    cfg.classify_mode = 3
    assert lib.lbm_init(ctypes.byref(cfg), ctypes.byref(bufs), ctypes.byref(ctx)) == B.LBM_EINVAL
    assert b"classify_mode" in lib.lbm_last_error(None)


def test_init_rejects_unknown_force_sum(lib):
    bufs = B.LbmBuffers()
    ctx = ctypes.c_void_p()
    cfg = _cfg()
    cfg.force_sum = 2
    assert lib.lbm_init(ctypes.byref(cfg), ctypes.byref(bufs), ctypes.byref(ctx)) == B.LBM_EINVAL
    assert b"force_sum" in lib.lbm_last_error(None)


def test_init_rejects_unknown_treatment_bits(lib):
    bufs = B.LbmBuffers()
    ctx = ctypes.c_void_p()
    cfg = _cfg()
    cfg.treatments = 16
    assert lib.lbm_init(ctypes.byref(cfg), ctypes.byref(bufs), ctypes.byref(ctx)) == B.LBM_EINVAL
    assert b"treatment" in lib.lbm_last_error(None)


def test_query_sizes_follow_the_lattice(lib):
    for lattice, q in ((0, 19), (19, 19), (15, 15)):
        cfg = _cfg()
        cfg.lattice = lattice
        s = B.lbm_query_sizes(cfg)
        es = 4
        assert s.population_bytes == q * s.cell_stride * es
        assert s.adjoint_bytes == q * s.cell_stride * 4
    cfg = _cfg()
    cfg.lattice = 27
    with pytest.raises(B.LbmError) as e:
        B.lbm_query_sizes(cfg)
    assert e.value.code == B.LBM_EINVAL
    assert b"lattice" in lib.lbm_last_error(None)


def test_query_sizes_rejects_bad_input(lib):
    with pytest.raises(B.LbmError) as e:
        B.lbm_query_sizes(_cfg(dims=(0, 4, 4)))
    assert e.value.code == B.LBM_EINVAL
    with pytest.raises(B.LbmError) as e:
        B.lbm_query_sizes(_cfg(storage=7))
    assert e.value.code == B.LBM_EINVAL


def test_init_rejects_bad_arguments_before_touching_the_device(lib):
    bufs = B.LbmBuffers()
    ctx = ctypes.c_void_p()
    for cfg in (_cfg(tau=0.5), _cfg(), _cfg(n_particles=2, box_half=7, dims=(16, 16, 16))):
        rc = lib.lbm_init(ctypes.byref(cfg), ctypes.byref(bufs), ctypes.byref(ctx))
        assert rc == B.LBM_EINVAL
        assert lib.lbm_last_error(None)
    # a periodic axis too short for the particle box
    fake = (B._P * 2)(1, 2)
    bufs = B.LbmBuffers(fake, fake, 3, 4)
    cfg = _cfg(n_particles=1, box_half=6, dims=(16, 40, 40), periodic=(1, 0, 0))
    assert lib.lbm_init(ctypes.byref(cfg), ctypes.byref(bufs), ctypes.byref(ctx)) == B.LBM_EINVAL
    assert b"2*box_half" in lib.lbm_last_error(None)


def test_calls_reject_a_null_context_without_touching_the_device(lib):
    """Every call on the hot path, the asynchronous classification and the
    synchronisation that reports its latched errors return EINVAL for a null
    context before any device work."""
    p = B.LbmParticles()
    prm = B.DemParams()
    assert lib.lbm_classify_nodes(None, ctypes.byref(p), None) == B.LBM_EINVAL
    assert lib.lbm_classify_nodes_async(None, ctypes.byref(p)) == B.LBM_EINVAL
    assert lib.lbm_step(None, ctypes.byref(p)) == B.LBM_EINVAL
    assert lib.dem_step(None, ctypes.byref(p), 1, ctypes.c_double(0.1), ctypes.byref(prm)) == B.LBM_EINVAL
    assert lib.lbm_synchronize(None) == B.LBM_EINVAL
    assert b"null context" in lib.lbm_last_error(None)
    n, tag = ctypes.c_size_t(), ctypes.c_uint64()
    assert lib.lbm_geometry_bytes(None, ctypes.byref(n), ctypes.byref(tag)) == B.LBM_EINVAL
    assert lib.lbm_geometry_save(None, None) == B.LBM_EINVAL
    assert lib.lbm_geometry_load(None, None, 0, ctypes.byref(p)) == B.LBM_EINVAL


# the binding's ctypes mirrors of the header's structs, field by field
STRUCTS = {
    "lbm_config": B.LbmConfig, "lbm_sizes": B.LbmSizes, "lbm_buffers": B.LbmBuffers,
    "lbm_particles": B.LbmParticles, "lbm_counts": B.LbmCounts, "dem_params": B.DemParams,
    "lbm_profile": B.LbmProfile,
}


def test_binding_structs_match_the_header_layout(tmp_path):
    """Compile a C program against include/mdlbm.h that prints sizeof and
    every field's offsetof, and compare with the ctypes structures."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "mdlbm.h"', "int main(void) {"]
    for cname, py in STRUCTS.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", f"-I{ROOT / 'include'}", str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, py in STRUCTS.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)

