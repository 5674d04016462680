"""Host-side checks of the C-ABI library that need no GPU: it loads, exports
every symbol include/*.h declares, sizes workspaces, and rejects invalid
input before touching the device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("tlb.h", "tlb3d.h")]
LIB = os.path.join(ROOT, "paper_1710_09534_amd", "libtlb.so")


def declared_symbols():
    out = set()
    for h in HEADERS:
        src = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        out |= set(re.findall(r"\b(tlb3?_[a-z0-9_]+)\s*\(", src))
    return sorted(out)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        import paper_1710_09534_amd.build as b
        b.build()
    return C.CDLL(LIB)


def test_exports_every_declared_symbol(lib):
    syms = declared_symbols()
    assert len(syms) >= 45 and any(s.startswith("tlb3_") for s in syms)
    for s in syms:
        assert hasattr(lib, s), s


def test_binding_names_match_header():
    from paper_1710_09534_amd import tlb
    for s in declared_symbols():
        assert s in tlb._SIGS or s.startswith("tlb_server"), s


def test_workspace_sizes():
    from paper_1710_09534_amd import tlb
    b64 = tlb.tlb_workspace_bytes(1024, 2048, tlb.TLB_FP64)
    b32 = tlb.tlb_workspace_bytes(1024, 2048, tlb.TLB_FP32)
    b16 = tlb.tlb_workspace_bytes(1024, 2048, tlb.TLB_FP16DEV)
    n = 1024 * 2048
    # two lattices of 27 planes + 4 history planes + staging
    assert b64 >= n * (2 * 27 * 8 + 4 * 8)
    assert b32 >= n * (2 * 27 * 4 + 4 * 4)
    assert b16 >= n * (2 * (25 * 2 + 2 * 4) + 4 * 4)
    assert b64 > b32 > b16 > 0
    assert tlb.tlb_workspace_bytes(2, 10, tlb.TLB_FP64) == 0
    assert tlb.tlb_workspace_bytes(10, 10, 7) == 0


def _fl(**kw):
    from paper_1710_09534_amd import workloads as W
    fl = W.fluid()
    fl.update(kw)
    return fl


@pytest.mark.parametrize("kw,code", [
    (dict(tau1=0.5), -2),
    (dict(sigma12=5e-3), -2),             # lambda_3 < 0
    (dict(sigma12=1.9e-3, sigma13=1e-3, sigma23=1e-3), -2),  # lambda_3 <= lambda_T/2
    (dict(D=0.0), -2),
    (dict(M0=-1.0), -2),
    (dict(rho=[1.0, 0.0, 1.0]), -2),
])
def test_create_rejects_inadmissible_parameters(kw, code):
    from paper_1710_09534_amd import tlb
    f = tlb.make_fluid(_fl(**kw))
    h = C.c_void_p()
    ws = C.c_void_p(1 << 20)  # never dereferenced: validation fails first
    st = tlb.lib.tlb_create(64, 64, 0, C.byref(f), ws, 1 << 40, None, C.byref(h))
    assert st == code and not h.value
    assert len(tlb.tlb_last_error()) > 0


def test_create_rejects_bad_sizes_and_pointers():
    from paper_1710_09534_amd import tlb
    f = tlb.make_fluid(_fl())
    h = C.c_void_p()
    assert tlb.lib.tlb_create(2, 64, 0, C.byref(f), C.c_void_p(256), 1 << 40, None,
                              C.byref(h)) == tlb.TLB_EINVAL
    assert tlb.lib.tlb_create(64, 64, 0, None, C.c_void_p(256), 1 << 40, None,
                              C.byref(h)) == tlb.TLB_EINVAL
    assert tlb.lib.tlb_create(64, 64, 0, C.byref(f), None, 1 << 40, None,
                              C.byref(h)) == tlb.TLB_EINVAL
    assert tlb.lib.tlb_create(64, 64, 0, C.byref(f), C.c_void_p(257), 1 << 40, None,
                              C.byref(h)) == tlb.TLB_EINVAL       # misaligned
    assert tlb.lib.tlb_create(64, 64, 0, C.byref(f), C.c_void_p(256), 1024, None,
                              C.byref(h)) == tlb.TLB_ENOMEM       # too small
    assert tlb.lib.tlb_create(64, 64, 9, C.byref(f), C.c_void_p(256), 1 << 40, None,
                              C.byref(h)) == tlb.TLB_EINVAL


def test_null_context_calls_fail_cleanly():
    from paper_1710_09534_amd import tlb
    out = np.zeros(3)
    assert tlb.lib.tlb_step(None, 1) == tlb.TLB_EINVAL
    assert tlb.lib.tlb_mass(None, tlb._dp(out)) == tlb.TLB_EINVAL
    assert tlb.lib.tlb_step_count(None) == -1
    tlb.lib.tlb_destroy(None)


def test_workspace_sizes_3d():
    from paper_1710_09534_amd import tlb
    n = 64 * 48 * 40
    b64 = int(tlb.lib.tlb3_workspace_bytes(64, 48, 40, tlb.TLB_FP64))
    b32 = int(tlb.lib.tlb3_workspace_bytes(64, 48, 40, tlb.TLB_FP32))
    # two lattices of 57 planes + 5 history + 2 c + 3 mu planes
    assert b64 >= n * (2 * 57 + 10) * 8
    assert b32 >= n * (2 * 57 + 10) * 4
    assert int(tlb.lib.tlb3_workspace_bytes(64, 48, 40, tlb.TLB_FP16DEV)) == 0
    assert int(tlb.lib.tlb3_workspace_bytes(64, 2, 40, tlb.TLB_FP64)) == 0


def test_create3_rejections():
    from paper_1710_09534_amd import tlb
    fl = tlb.make_fluid(_fl())
    h = C.c_void_p()
    ws = (C.c_uint8 * 512)()
    st = tlb.lib.tlb3_create(16, 16, 16, tlb.TLB_FP16DEV, C.byref(fl), 0.0, C.cast(ws, C.c_void_p),
                             512, None, C.byref(h))
    assert st == tlb.TLB_EINVAL
    st = tlb.lib.tlb3_create(16, 16, 16, tlb.TLB_FP64, C.byref(fl), 0.0, C.cast(ws, C.c_void_p),
                             512, None, C.byref(h))
    assert st in (tlb.TLB_EINVAL, tlb.TLB_ENOMEM)
    assert not h.value


def _max_rows(nx, elem, hist_elem, planes=9):
    """Largest ny whose padded family of `planes` planes and 4-plane history
    stay below 2 GiB (rows padded to a multiple of 64 nodes)."""
    pitch = -(-nx // 64) * 64
    lim = (1 << 31) - 1
    return min(lim // (planes * pitch * elem), lim // (4 * pitch * hist_elem))


@pytest.mark.parametrize("prec,nx,elem,hist", [(0, 5430, 8, 8), (1, 7710, 4, 4), (2, 7650, 4, 4)])
def test_size_limit_boundary(prec, nx, elem, hist):
    """tlb_workspace_bytes is non-zero up to the largest lattice tlb_create
    accepts and 0 one row beyond it; tlb_create agrees."""
    from paper_1710_09534_amd import tlb
    ny = _max_rows(nx, elem, hist)
    assert tlb.tlb_workspace_bytes(nx, ny, prec) > 0
    assert tlb.tlb_workspace_bytes(nx, ny + 1, prec) == 0
    f = tlb.make_fluid(_fl())
    h = C.c_void_p()
    assert tlb.lib.tlb_create(nx, ny + 1, prec, C.byref(f), C.c_void_p(256), 1 << 40, None,
                              C.byref(h)) == tlb.TLB_EINVAL


def test_workspace_is_lattice_plus_modest_staging():
    """The staging area holds the 4 init fields, not a full copy of the
    populations: workspace bytes per node stay close to the lattice's own
    (two population buffers, the history planes of each, the material byte)."""
    from paper_1710_09534_amd import tlb
    n = 1024 * 2048
    for prec, lattice in ((0, 2 * 27 * 8 + 2 * 4 * 8 + 1), (1, 2 * 27 * 4 + 2 * 4 * 4 + 1),
                          (2, 2 * (16 * 2 + 11 * 4) + 2 * 4 * 4 + 1)):
        per_node = tlb.tlb_workspace_bytes(1024, 2048, prec) / n
        assert lattice <= per_node <= lattice + 4 * 8 + 1, (prec, per_node)


def test_size_limit_boundary_3d():
    from paper_1710_09534_amd import tlb
    for prec, elem in ((0, 8), (1, 4)):
        nx, ny = 200, 150                      # pitch 256
        nz = ((1 << 31) - 1) // (19 * 256 * ny * elem)
        assert tlb.lib.tlb3_workspace_bytes(nx, ny, nz, prec) > 0
        assert tlb.lib.tlb3_workspace_bytes(nx, ny, nz + 1, prec) == 0
    assert tlb.lib.tlb3_workspace_bytes(64, 64, 65536, 1) == 0
