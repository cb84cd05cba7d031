"""The C ABI library loads, exports every entry point include/pic.h declares,
and rejects invalid arguments before touching a GPU.  CPU only."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pic.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pic_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    import paper_2605_05469_amd as P
    if not os.path.exists(P.LIB_PATH):
        from paper_2605_05469_amd import build
        build.build()
    return P.lib()


def test_header_declares_the_hot_path():
    names = _declared()
    for n in ("pic_deposit_cic", "pic_poisson_pcg", "pic_gather_push", "pic_step"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    import paper_2605_05469_amd as P
    out = subprocess.run(["nm", "-D", "--defined-only", P.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (pic_[a-z_0-9]+)", out))
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing
    assert set(P.EXPORTS) <= exported


def test_abi_version_and_errors_without_gpu(lib):
    import paper_2605_05469_amd as P
    assert lib.pic_abi_version() == 3
    p = P.landau_params(32, 8)
    assert lib.pic_workspace_bytes(ctypes.byref(p)) > 3 * 8 * 32 ** 3
    h = ctypes.c_void_p()
    for field, bad in (("n", 33), ("n", 16), ("n", 2048), ("rtol", 0.0), ("length", -1.0),
                       ("solver", 7), ("np_max", -5), ("flags", 256),
                       ("ssor_omega", 2.5), ("ssor_inner", -1), ("bc", 3), ("bc", -1)):
        q = P.landau_params(32, 8)
        setattr(q, field, bad)
        assert lib.pic_workspace_bytes(ctypes.byref(q)) == 0
        assert lib.pic_create(ctypes.byref(q), ctypes.byref(h)) == P.PIC_ERR_INVALID
        assert lib.pic_last_error()
    # bounded boxes take only the stencil solver forms
    for bc, solver in ((P.BC_DIRICHLET, "fft"), (P.BC_NEUMANN, "fcg_learned")):
        q = P.landau_params(32, 8, solver=solver, bc=bc)
        assert lib.pic_create(ctypes.byref(q), ctypes.byref(h)) == P.PIC_ERR_INVALID
    assert lib.pic_create(None, ctypes.byref(h)) == P.PIC_ERR_INVALID
    assert lib.pic_destroy(None) == 0
    # the entry points reject a NULL context instead of crashing
    assert lib.pic_poisson_pcg(None, None, None, None, None, None, None, None) == P.PIC_ERR_INVALID
    assert lib.pic_gather_push(None, 0, *([None] * 10), None) == P.PIC_ERR_INVALID
    assert lib.pic_deposit_cic(None, 0, None, None, None, None, None, None, None) == P.PIC_ERR_INVALID
    assert lib.pic_set_flags(None, 0) == P.PIC_ERR_INVALID
    # the no-allocation deposit refuses grids beyond its static scratch
    for n in (128, 16, 33):
        q = P.landau_params(n, 1)
        assert lib.pic_deposit_cic_noalloc(ctypes.byref(q), 0, None, None, None, None, None, None,
                                           None) == P.PIC_ERR_INVALID
        assert b"n must be" in lib.pic_last_error()
    assert lib.pic_deposit_cic_noalloc(None, 0, *([None] * 7)) == P.PIC_ERR_INVALID


def test_single_hip_runtime_is_loaded(lib):
    maps = open("/proc/self/maps").read()
    hips = {l.split()[-1] for l in maps.splitlines() if "libamdhip64" in l}
    assert len(hips) == 1, hips
