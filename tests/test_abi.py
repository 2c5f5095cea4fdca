"""The C-ABI library loads, exports every function include/lbib.h declares, lays out its
structs as a C compiler does, and rejects bad arguments on the host before touching the
GPU.  CPU only: no compute call is made."""
import ctypes as C
import os
import re
import subprocess

import pytest

from paper_1808_01448_amd import lbib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbib.h")


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(lbib.LIB_PATH):
        from paper_1808_01448_amd import build

        build.build()
    return lbib.lib()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbib_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(L):
    names = declared_functions()
    assert len(names) >= 29
    for n in names:
        assert hasattr(L, n), n
    assert sorted(lbib.EXPORTED) == names


def test_abi_version(L):
    assert L.lbib_abi_version() == 2


def test_struct_layout_matches_c(tmp_path):
    """Compile a probe with gcc against the header and compare sizes and offsets with the
    ctypes mirrors of the binding."""
    structs = {
        "lbib_lattice_desc": lbib.LatticeDesc, "lbib_particle_desc": lbib.ParticleDesc,
        "lbib_ligand_desc": lbib.LigandDesc, "lbib_receptor_desc": lbib.ReceptorDesc,
        "lbib_particle_state": lbib.ParticleState, "lbib_request_result": lbib.RequestResult,
    }
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "lbib.h"', "int main(void){"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0;}")
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe)]).decode().split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, py in structs.items():
        assert got[(cname, "size")] == C.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


FAKE_STREAM = C.c_void_p(0x1)  # never dereferenced: nothing is enqueued before lbib_init


def _create(L, **kw):
    d = lbib.LatticeDesc(kw.get("nx", 64), kw.get("ny", 32), kw.get("tau", 0.8), kw.get("re", 0.1),
                         kw.get("drive", 0), kw.get("precision", 0), 0)
    h = C.c_void_p()
    st = L.lbib_create(C.byref(d), FAKE_STREAM, C.byref(h))
    return st, h


@pytest.mark.parametrize("kw,status", [
    (dict(nx=3), lbib.E_INVALID), (dict(ny=2), lbib.E_INVALID), (dict(tau=0.5), lbib.E_INVALID),
    (dict(tau=float("nan")), lbib.E_INVALID), (dict(re=-1.0), lbib.E_INVALID),
    (dict(drive=2), lbib.E_INVALID), (dict(drive=-1), lbib.E_INVALID), (dict(precision=6), lbib.E_UNSUPPORTED), (dict(precision=-1), lbib.E_UNSUPPORTED),
])
def test_create_rejects(L, kw, status):
    st, h = _create(L, **kw)
    assert st == status
    assert L.lbib_last_error(None)


def _pdesc(**kw):
    d = dict(shape=0, a_major=5.0, b_minor=5.0, xc=20.0, yc=10.0, theta0=0.0, rho_p=1.0, n_markers=32)
    d.update(kw)
    return lbib.ParticleDesc(**d)


@pytest.mark.parametrize("kw", [
    dict(shape=2), dict(a_major=-1.0), dict(n_markers=7), dict(n_markers=2000), dict(rho_p=0.0),
    dict(yc=4.4), dict(yc=27.0), dict(a_major=30.0, yc=15.0), dict(n_markers=200),
    dict(shape=1, b_minor=0.0), dict(xc=float("inf")),
])
def test_particle_validation(L, kw):
    st, h = _create(L)
    assert st == lbib.OK
    try:
        pid = C.c_int32(-7)
        assert L.lbib_particle_add(h, C.byref(_pdesc(**kw)), C.byref(pid)) == lbib.E_INVALID
        assert pid.value == -7
        assert L.lbib_last_error(h)
    finally:
        L.lbib_destroy(h)


def test_call_order_and_ligand_validation(L):
    st, h = _create(L)
    try:
        pid = C.c_int32()
        assert L.lbib_step(h, 1) == lbib.E_STATE
        assert L.lbib_particle_add(h, C.byref(_pdesc()), C.byref(pid)) == lbib.OK and pid.value == 0
        assert L.lbib_particle_add(h, C.byref(_pdesc(xc=40.0)), C.byref(pid)) == lbib.OK and pid.value == 1
        # a particle without ligands cannot be initialised
        assert L.lbib_init(h) == lbib.E_STATE
        bad = lbib.LigandDesc(3, 2, 27.8, 0.5, 6.8e-3, 0.5, 1.0, 1e-4, 1e-5, 1e-8)
        assert L.lbib_ligands_set(h, 0, C.byref(bad)) == lbib.E_INVALID
        bad = lbib.LigandDesc(1, 2, 27.8, 0.5, 6.8e-3, 0.5, 1.0, 1e-4, 0.0, 1e-8)
        assert L.lbib_ligands_set(h, 0, C.byref(bad)) == lbib.E_INVALID
        assert L.lbib_ligands_set(h, 5, C.byref(bad)) == lbib.E_INVALID
        good = lbib.LigandDesc(1, 2, 27.8, 0.5, 6.8e-3, 0.5, 1.0, 1e-4, 1e-5, 1e-8)
        assert L.lbib_ligands_set(h, 0, C.byref(good)) == lbib.OK
        assert L.lbib_init(h) == lbib.E_STATE  # particle 1 still has no ligands
        assert L.lbib_ligands_set(h, 1, C.byref(good)) == lbib.OK
        assert L.lbib_receptors_set(h, C.byref(lbib.ReceptorDesc(0, 0.5))) == lbib.E_UNSUPPORTED
        assert L.lbib_receptors_set(h, C.byref(lbib.ReceptorDesc(1, 1.0))) == lbib.E_UNSUPPORTED
        assert L.lbib_receptors_set(h, C.byref(lbib.ReceptorDesc(0, 1.0))) == lbib.OK
        s = lbib.ParticleState()
        assert L.lbib_read_particle(h, 0, C.byref(s)) == lbib.E_STATE
        assert L.lbib_step(h, -1) == lbib.E_INVALID
    finally:
        L.lbib_destroy(h)
    L.lbib_destroy(None)


def test_kernel_entry_points_validate_sizes(L):
    assert L.lbib_kernel_philox(None, None, None, -1, None) == lbib.E_INVALID
    assert L.lbib_kernel_mls(None, 1, 64, 32, None, None, None, None, None) == lbib.E_INVALID
    assert L.lbib_kernel_mls(None, 0, 2, 32, None, None, None, None, None) == lbib.E_INVALID
    p = (C.c_double * 7)()
    assert L.lbib_kernel_bonds(None, None, None, None, None, None, None, 0, 1, p, 0, 0, None) == lbib.E_INVALID
    v = C.c_double()
    assert L.lbib_bandwidth_probe(17, 1, None, C.byref(v)) == lbib.E_INVALID


def test_pool_host_validation(L):
    h = C.c_void_p()
    assert L.lbib_pool_create(9, 1 << 30, 16, FAKE_STREAM, C.byref(h)) == lbib.E_UNSUPPORTED
    assert L.lbib_pool_create(1, 0, 16, FAKE_STREAM, C.byref(h)) == lbib.E_INVALID
    assert L.lbib_pool_create(1, 1 << 30, 0, FAKE_STREAM, C.byref(h)) == lbib.E_INVALID
    assert L.lbib_pool_create(1, 1 << 30, 70000, FAKE_STREAM, C.byref(h)) == lbib.E_INVALID
    assert L.lbib_pool_last_error(None)
    assert h.value is None
    assert L.lbib_pool_step(None, 1) == lbib.E_INVALID
    n = C.c_int32()
    assert L.lbib_pool_poll(None, None, 0, C.byref(n)) == lbib.E_INVALID
    assert L.lbib_pool_remove(None, 0) == lbib.E_INVALID
    L.lbib_pool_destroy(None)


def test_pool_footprint(L):
    """Two population buffers of nine population rows per lattice row (each padded to 256
    bytes), plus three FP32 moment rows for the f - f_eq storages, plus the particle's
    buffers; refused for descriptors lbib_create / lbib_particle_add would refuse."""
    def fp(nx, ny, prec, **kw):
        d = lbib.LatticeDesc(nx, ny, 0.8, 0.1, 0, prec, 0)
        v = C.c_int64(-1)
        st = L.lbib_pool_footprint(C.byref(d), C.byref(_pdesc(**kw)), C.byref(v))
        return st, v.value

    for nx, ny, prec, elem in [(64, 32, 1, 4), (100, 40, 1, 4), (100, 40, 0, 8), (1000, 300, 1, 4)]:
        st, v = fp(nx, ny, prec)
        assert st == lbib.OK
        pitch = -(-nx * elem // 256) * 256 // elem
        pop = 2 * 9 * pitch * ny * elem
        assert pop < v < pop + 200_000, (nx, ny, prec, v - pop)
    # (1000 x 300: the moment rows, 7.4 MB, far exceed the particle's share)
    for nx, ny, prec in [(100, 40, 2), (100, 40, 4), (1000, 300, 2), (1000, 300, 4), (1000, 300, 5)]:
        st, v = fp(nx, ny, prec)
        assert st == lbib.OK
        row = -(-nx * 2 // 256) * 256 // 2
        pop = 2 * (9 * row * ny * 2 + (3 * row * ny * 4 if prec >= 4 else 0))
        assert pop < v < pop + 200_000, (nx, ny, prec, v - pop)
    # more markers or a larger particle never cost less
    assert fp(64, 32, 1, n_markers=64)[1] > fp(64, 32, 1)[1]
    assert fp(200, 64, 1, a_major=20.0, yc=30.0)[1] > fp(200, 64, 1)[1]
    assert fp(64, 32, 1, n_markers=7)[0] == lbib.E_INVALID
    assert fp(3, 32, 1)[0] == lbib.E_INVALID


def test_server_host_validation(L):
    h = C.c_void_p()
    assert L.lbib_server_create(1, 1 << 30, 16, 0, 0, FAKE_STREAM, C.byref(h)) == lbib.E_INVALID
    assert L.lbib_server_create(1, 1 << 30, 16, 10, -1, FAKE_STREAM, C.byref(h)) == lbib.E_INVALID
    assert L.lbib_server_create(7, 1 << 30, 16, 10, 0, FAKE_STREAM, C.byref(h)) == lbib.E_UNSUPPORTED
    assert L.lbib_server_last_error(None)
    assert L.lbib_server_progress(None, None) == lbib.E_INVALID
    L.lbib_server_destroy(None)


def test_particle_count_limit(L):
    st, h = _create(L, nx=256)
    try:
        pid = C.c_int32()
        for k in range(64):
            assert L.lbib_particle_add(h, C.byref(_pdesc(xc=4.0 * k)), C.byref(pid)) == lbib.OK and pid.value == k
        assert L.lbib_particle_add(h, C.byref(_pdesc()), C.byref(pid)) == lbib.E_UNSUPPORTED
    finally:
        L.lbib_destroy(h)


def test_static_solve_host_validation(L):
    """lbib_solve_static checks its arguments before touching the GPU: a NULL descriptor, a
    negative step count, a particle outside the channel, an unaligned or too small population
    buffer and a particle whose buffers exceed the 8 MiB static area are refused; with no
    population buffer it reports the bytes the lattice needs (two population buffers)."""
    from paper_1808_01448_amd import workloads as W

    w = W.channel_small_fp64()
    lat = lbib._lattice_desc(w["lattice"])
    part = lbib._particle_desc(w["particle"])
    lig = lbib._ligand_desc(w["ligand"])
    v = C.c_int64(0)
    assert L.lbib_solve_static(None, C.byref(part), C.byref(lig), 10, None, C.byref(v), None, None, None) == lbib.E_INVALID
    assert L.lbib_solve_static(C.byref(lat), C.byref(part), C.byref(lig), -1, None, C.byref(v), None, None,
                               None) == lbib.E_INVALID
    assert L.lbib_solve_static(C.byref(lat), C.byref(part), C.byref(lig), 10, None, C.byref(v), None, None,
                               None) == lbib.OK
    nx, ny = w["lattice"]["nx"], w["lattice"]["ny"]
    assert v.value == 2 * 9 * nx * ny * 8  # FP64 rows of 256 x 8 bytes need no padding
    bad = lbib._particle_desc(dict(w["particle"], yc=-5.0))
    assert L.lbib_solve_static(C.byref(lat), C.byref(bad), C.byref(lig), 10, None, C.byref(v), None, None,
                               None) == lbib.E_INVALID
    small = C.c_int64(16)
    assert L.lbib_solve_static(C.byref(lat), C.byref(part), C.byref(lig), 10, C.c_void_p(4096), C.byref(small),
                               None, None, None) == lbib.E_INVALID
    assert b"needs" in L.lbib_last_error(None)
    enough = C.c_int64(1 << 30)
    assert L.lbib_solve_static(C.byref(lat), C.byref(part), C.byref(lig), 10, C.c_void_p(4096 + 8), C.byref(enough),
                               None, None, None) == lbib.E_INVALID
    assert b"aligned" in L.lbib_last_error(None)
    big = W.channel_small_fp64()
    big["lattice"].update(nx=1024, ny=1024)
    big["particle"].update(a_major=200.0, b_minor=200.0, xc=512.0, yc=220.0, n_markers=1024)
    assert L.lbib_solve_static(C.byref(lbib._lattice_desc(big["lattice"])), C.byref(lbib._particle_desc(big["particle"])),
                               C.byref(lig), 10, None, C.byref(v), None, None, None) == lbib.E_INVALID
    assert b"static area" in L.lbib_last_error(None)


def test_server_read_outs_validate(L):
    """The server's trace and bond read-outs refuse a NULL handle, an unknown request and bad
    capacities without touching the GPU."""
    n = C.c_int64()
    assert L.lbib_server_set_trace(None, 10) == lbib.E_INVALID
    assert L.lbib_server_read_trace(None, 0, None, 0, C.byref(n)) == lbib.E_INVALID
    assert L.lbib_server_read_bonds(None, 0, None, None, 64) == lbib.E_INVALID
