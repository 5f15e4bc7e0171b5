"""CPU-side checks of the C ABI library: it loads, exports every entry point
the public header declares, and its host-only validation returns the
documented codes.  No device work runs here."""
import ctypes as ct
import os
import re

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hemelb_hip.h")


@pytest.fixture(scope="module")
def hl():
    import paper_2010_04144_amd as hl
    hl.lib()
    return hl


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hl_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol(hl):
    names = declared_functions()
    assert len(names) >= 35
    lib = ct.CDLL(hl._lib.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(names) == set(hl._lib.SIGNATURES), set(names) ^ set(hl._lib.SIGNATURES)


def test_status_strings(hl):
    for code in (0, -1, -2, -3, -4, -5, -6, 1, 2):
        s = hl.status_string(code)
        assert s and s != "unknown status"
    assert hl.status_string(12345) == "unknown status"


def test_validate_accepts_generated_geometries(hl):
    for g in (synth.cylinder(), synth.tubes(3), synth.cylinder(nz=4, ends="periodic"),
              synth.tree_geometry(3, 6.0, 1, lam=6.0)):
        assert hl.hl_validate_sites(g.nbr, len(g.iolets)) == hl.HL_OK


def test_branching_artery_recipe(hl):
    """The benchmark workload: a seeded Murray tree of depth 8 and root radius
    40 in a 768^3 box, with the segment length fitted so the tree fits
    (lambda = 3.7114), gives 6,064,894 sites, one root inlet and 256 leaf
    outlets, and 4,716,345 wall links, each with a wall fraction in (0, 1];
    its site list passes the library's host checks."""
    geo = synth.branching_artery(box=768)
    assert geo.n == 6064894
    assert abs(geo.meta["lam"] - 3.7114) < 1e-4
    kinds = [io.kind for io in geo.iolets]
    assert kinds[0] == "inlet" and kinds.count("outlet") == 256 and len(kinds) == 257
    assert int(np.count_nonzero(geo.nbr == -1)) == 4716345 == geo.q.size
    assert float(geo.q.min()) > 0.0 and float(geo.q.max()) <= 1.0
    assert hl.hl_validate_sites(geo.nbr, len(geo.iolets)) == hl.HL_OK


def test_validate_rejects_malformed_lists(hl):
    g = synth.cylinder(nz=6)
    n = g.n
    nbr = g.nbr.copy()
    nbr[0, 3] = 4                              # rest entry must be the site itself
    assert hl.hl_validate_sites(nbr, 2) == hl.HL_E_RANGE
    nbr = g.nbr.copy()
    nbr[1, 10] = n + 5                          # index beyond the list
    assert hl.hl_validate_sites(nbr, 2) == hl.HL_E_RANGE
    nbr = g.nbr.copy()
    nbr[1, 10] = -2 - 7                         # unknown iolet code
    assert hl.hl_validate_sites(nbr, 2) == hl.HL_E_RANGE
    nbr = g.nbr.copy()
    s = int(np.flatnonzero(nbr[1] >= 0)[0])
    nbr[1, s] = int(np.flatnonzero(nbr[1] >= 0)[5])   # link whose reverse does not come back
    assert hl.hl_validate_sites(nbr, 2) == hl.HL_E_INVAL
    nbr = g.nbr.copy()
    inl = int(np.flatnonzero((nbr == -2).any(0))[0])
    k = int(np.flatnonzero(nbr[:, inl] == -1)[0]) if (nbr[:, inl] == -1).any() else 1
    nbr[k, inl] = -3                            # same site borders inlet and outlet
    assert hl.hl_validate_sites(nbr, 2) == hl.HL_E_INVAL


def test_validate_edge_sizes(hl):
    empty = np.zeros((19, 0), np.int32)
    assert hl.hl_validate_sites(empty, 0) == hl.HL_OK
    one = np.full((19, 1), -1, np.int32)
    one[0, 0] = 0
    assert hl.hl_validate_sites(one, 0) == hl.HL_OK
    lib = hl.lib()
    assert lib.hl_validate_sites(-1, None, 0) == hl.HL_E_RANGE
    assert lib.hl_validate_sites(2**31, None, 0) == hl.HL_E_RANGE


def test_create_without_a_device_fails_cleanly(hl):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ct.c_void_p()
    assert hl.lib().hl_create(ct.byref(h), 0, hl.HL_F64, 0) == hl.HL_E_DEVICE
    assert not h.value
    with pytest.raises(hl.HLError):
        hl.Context(0, "f64")


def test_bad_arguments_rejected_before_device(hl):
    lib = hl.lib()
    h = ct.c_void_p()
    assert lib.hl_create(ct.byref(h), 0, 7, 0) == hl.HL_E_INVAL
    assert lib.hl_create(ct.byref(h), 0, 0, 1 << 12) == hl.HL_E_INVAL
    assert lib.hl_create(ct.byref(h), 0, 0, hl.HL_ORDER_BRICK_32) == hl.HL_E_INVAL  # needs HL_ORDER_BRICK
    assert lib.hl_create(None, 0, 0, 0) == hl.HL_E_INVAL
    lib.hl_destroy(None)


def test_every_context_call_rejects_a_null_context(hl):
    """Each call of the header that takes a context returns HL_E_INVAL for a
    NULL one (the other arguments NULL or 0), without a device."""
    lib = hl.lib()
    with open(HEADER) as fh:
        names = re.findall(r"^int (hl_\w+)\(hl_ctx \*ctx", fh.read(), flags=re.M)
    assert len(names) >= 30
    bad = {}
    for nm in names:
        f = getattr(lib, nm)
        args = [None]
        for t in f.argtypes[1:]:
            ptr = t in (ct.c_void_p, ct.c_char_p) or (isinstance(t, type) and issubclass(t, ct._Pointer))
            args.append(None if ptr else 0)
        rc = f(*args)
        if rc != hl.HL_E_INVAL:
            bad[nm] = rc
    assert not bad, bad

def test_copy_bandwidth_argument_checks(hl):
    """The copy-ceiling call rejects bad arguments on the host, before any
    device call (the pointers below are never touched)."""
    lib = hl.lib()
    out = ct.c_double(-1.0)
    P = ct.c_void_p
    a, b = P(1 << 20), P(1 << 30)
    assert lib.hl_copy_bandwidth(None, a, 64, 1, None, ct.byref(out)) == hl.HL_E_INVAL
    assert lib.hl_copy_bandwidth(b, None, 64, 1, None, ct.byref(out)) == hl.HL_E_INVAL
    assert lib.hl_copy_bandwidth(b, a, 64, 1, None, None) == hl.HL_E_INVAL
    assert lib.hl_copy_bandwidth(b, a, 0, 1, None, ct.byref(out)) == hl.HL_E_INVAL
    assert lib.hl_copy_bandwidth(b, a, 40, 1, None, ct.byref(out)) == hl.HL_E_INVAL      # not whole 16-byte units
    assert lib.hl_copy_bandwidth(b, a, 64, 0, None, ct.byref(out)) == hl.HL_E_INVAL
    assert lib.hl_copy_bandwidth(b, a, 64, 1001, None, ct.byref(out)) == hl.HL_E_INVAL
    assert lib.hl_copy_bandwidth(P((1 << 30) + 8), a, 64, 1, None, ct.byref(out)) == hl.HL_E_INVAL  # misaligned
    assert lib.hl_copy_bandwidth(P((1 << 20) + 16), a, 64, 1, None, ct.byref(out)) == hl.HL_E_INVAL  # overlap
    assert lib.hl_copy_bandwidth(a, P((1 << 20) + 48), 64, 1, None, ct.byref(out)) == hl.HL_E_INVAL  # overlap
    # 2^44 bytes need 2^32 work-groups of 256 lanes: beyond the grid limit
    assert lib.hl_copy_bandwidth(P(1 << 52), a, 1 << 44, 1, None, ct.byref(out)) == hl.HL_E_RANGE
    assert out.value == -1.0


@pytest.mark.slow
def test_validate_site_list_beyond_2_31_entries():
    """A periodic box of 113,126,400 sites: its neighbour table holds
    2,149,401,600 entries (more than 2^31, the paper's BigCount limit of
    Sec. 2.1), which the host checks walk with 64-bit offsets; a broken
    reverse link near the end is still found.  About 9 GB of host memory."""
    import paper_2010_04144_amd as hl
    nx, ny, nz = 480, 480, 491
    n = nx * ny * nz
    assert 19 * n > 2 ** 31
    cx = [0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0]
    cy = [0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1]
    cz = [0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1]
    nbr = np.empty((19, n), dtype=np.int32)
    idx = np.arange(n, dtype=np.int32).reshape(nz, ny, nx)
    for i in range(19):
        nbr[i] = np.roll(idx, shift=(-cz[i], -cy[i], -cx[i]), axis=(0, 1, 2)).reshape(-1)
    del idx
    assert hl.hl_validate_sites(nbr, 0) == hl.HL_OK
    nbr[18, n - 7] = (nbr[18, n - 7] + 1) % n
    assert hl.hl_validate_sites(nbr, 0) == hl.HL_E_INVAL
