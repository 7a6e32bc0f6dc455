"""Host-side checks of the C ABI (no GPU): exported symbols, option validation,
the Table 1 pencil blocks (Sec. 3.1-3.2) and status codes.

The library's host entry points pf_check and pf_query_dims never touch the
GPU; pf_setup rejects bad arguments before it does.
"""
import os
import re
import subprocess

import pytest

import paper_1905_02803_amd as pf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pencilfft.h")
GOLDEN = os.path.join(ROOT, "tests", "golden", "table1_blocks.txt")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pf_\w+)\s*\(", text)))


def test_library_exports_every_declared_function():
    names = declared_functions()
    assert len(names) >= 15
    out = subprocess.run(["nm", "-D", "--defined-only", pf.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r" T (pf_\w+)$", out, flags=re.M))
    missing = [n for n in names if n not in exported]
    assert not missing, f"declared but not exported: {missing}"
    lib = pf.lib()
    for n in names:
        assert hasattr(lib, n)


def test_binding_mirrors_the_abi():
    assert sorted(pf.EXPORTED) == declared_functions()
    for n in pf.EXPORTED:
        assert callable(getattr(pf, n))


def test_layout_defaults():
    lay = pf.pf_layout_init()
    assert (lay.m1, lay.m2, lay.stride1, lay.useeven, lay.precision, lay.math, lay.inplace, lay.third) == \
        (1, 1, 1, 0, pf.PF_F32, pf.PF_PLAIN, 0, pf.PF_THIRD_FFT)


@pytest.mark.parametrize("shape", [(1024, 1024, 1024), (480, 360, 250), (32, 32, 32), (1, 1, 1), (49, 75, 243),
                                   (8192, 2, 3)])
def test_check_accepts_7_smooth_grids(shape):
    assert pf.pf_check(*shape) == pf.PF_OK


@pytest.mark.parametrize("shape,code", [
    ((0, 4, 4), pf.PF_EINVAL), ((4, -1, 4), pf.PF_EINVAL), ((4, 4, 0), pf.PF_EINVAL),
    ((11, 4, 4), pf.PF_EUNSUPPORTED), ((4, 13, 4), pf.PF_EUNSUPPORTED), ((4, 4, 17 * 2), pf.PF_EUNSUPPORTED),
    ((16384, 2, 2), pf.PF_EUNSUPPORTED),
])
def test_check_rejects(shape, code):
    assert pf.pf_check(*shape) == code


def test_f64_length_limit():
    assert pf.pf_check(4096, 4, 4, pf.Layout(precision=pf.PF_F64)) == pf.PF_OK
    assert pf.pf_check(8192, 4, 4, pf.Layout(precision=pf.PF_F64)) == pf.PF_EUNSUPPORTED


@pytest.mark.parametrize("lay,code", [
    # Eq. 2 read as: every block of every pencil non-empty (m1 <= min(nx/2+1, ny), m2 <= min(ny, nz))
    (dict(m1=5, m2=1), pf.PF_EINVAL),   # nx/2+1 = 5 for nx = 8 is fine, ny = 4 is not
    (dict(m1=4, m2=4), pf.PF_OK),
    (dict(m1=1, m2=5), pf.PF_EINVAL),   # nz = 6 fine, ny = 4 not
    (dict(m1=0), pf.PF_EINVAL),
    (dict(stride1=2), pf.PF_EINVAL),
    (dict(precision=7), pf.PF_EINVAL),
    (dict(math=9), pf.PF_EINVAL),
    (dict(inplace=3), pf.PF_EINVAL),
    (dict(third=5), pf.PF_EINVAL),
    (dict(useeven=2), pf.PF_EINVAL),
    # share-only: rank (r1, r2) must lie in the grid; r1, r2 must be 0 otherwise
    (dict(share_only=1, m1=2, m2=3, r1=1, r2=2), pf.PF_OK),
    (dict(share_only=1, m1=2, r1=2), pf.PF_EINVAL),
    (dict(share_only=1, m2=3, r2=-1), pf.PF_EINVAL),
    (dict(share_only=2), pf.PF_EINVAL),
    (dict(r1=1, m1=2), pf.PF_EINVAL),
])
def test_check_layout_values(lay, code):
    assert pf.pf_check(8, 4, 6, pf.Layout(**lay)) == code


def _blocks(nx, ny, nz, lay, pencil):
    return {(r1, r2): pf.pf_query_dims(nx, ny, nz, lay, pencil, r1, r2)
            for r1 in range(lay.m1) for r2 in range(lay.m2)}


@pytest.mark.parametrize("grid,m", [((24, 20, 18), (4, 6)), ((12, 10, 9), (2, 3)), ((30, 7, 10), (3, 2)),
                                    ((9, 6, 5), (5, 2))])
@pytest.mark.parametrize("stride1", [1, 0])
def test_blocks_tile_each_pencil_exactly_once(grid, m, stride1):
    nx, ny, nz = grid
    lay = pf.Layout(m1=m[0], m2=m[1], stride1=stride1)
    nxh = nx // 2 + 1
    for pencil, extent in ((pf.PF_PENCIL_X, (nx, ny, nz)), (pf.PF_PENCIL_Y, (nxh, ny, nz)),
                           (pf.PF_PENCIL_Z, (nxh, ny, nz))):
        cover = {}
        for (r1, r2), (st, sz, od) in _blocks(nx, ny, nz, lay, pencil).items():
            assert all(s > 0 for s in sz), (pencil, r1, r2, sz)
            for x in range(st[0], st[0] + sz[0]):
                for y in range(st[1], st[1] + sz[1]):
                    for z in range(st[2], st[2] + sz[2]):
                        assert (x, y, z) not in cover
                        cover[(x, y, z)] = (r1, r2)
        assert len(cover) == extent[0] * extent[1] * extent[2]


def test_table1_blocks_of_the_papers_uneven_examples():
    rows = [ln.split() for ln in open(GOLDEN) if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 48
    letters = "XYZ"
    for r in rows:
        nx, ny, nz, m1, m2, s1 = map(int, r[:6])
        pencil = {"X": pf.PF_PENCIL_X, "Y": pf.PF_PENCIL_Y, "Z": pf.PF_PENCIL_Z}[r[6]]
        r1, r2 = int(r[7]), int(r[8])
        L = tuple(map(int, r[9:12]))
        order = r[12]
        st, sz, od = pf.pf_query_dims(nx, ny, nz, pf.Layout(m1=m1, m2=m2, stride1=s1), pencil, r1, r2)
        assert tuple(sz[a] for a in od) == L, r
        assert "".join(letters[a] for a in od) == order, r


def test_query_dims_rejects_bad_rank_and_pencil():
    lay = pf.Layout(m1=2, m2=3)
    with pytest.raises(pf.PfError):
        pf.pf_query_dims(16, 16, 16, lay, pf.PF_PENCIL_X, 2, 0)
    with pytest.raises(pf.PfError):
        pf.pf_query_dims(16, 16, 16, lay, pf.PF_PENCIL_X, 0, 3)
    with pytest.raises(pf.PfError):
        pf.pf_query_dims(16, 16, 16, lay, 3, 0, 0)


def test_strerror_names_every_code():
    codes = [pf.PF_OK, pf.PF_EINVAL, pf.PF_EUNSUPPORTED, pf.PF_EALIGN, pf.PF_EALIAS, pf.PF_ENOMEM,
             pf.PF_EWORKSPACE, pf.PF_EHIP]
    names = [pf.pf_strerror(c) for c in codes]
    assert len(set(names)) == len(codes)
    assert pf.pf_strerror(-99) == "unknown error"


def test_setup_rejects_bad_arguments_before_touching_the_gpu():
    for shape, lay, code in [((0, 4, 4), pf.Layout(), pf.PF_EINVAL),
                             ((11, 4, 4), pf.Layout(), pf.PF_EUNSUPPORTED),
                             ((8, 4, 6), pf.Layout(m1=5), pf.PF_EINVAL),
                             ((8, 4, 6), pf.Layout(share_only=1, r1=1), pf.PF_EINVAL),
                             ((8, 4, 6), pf.Layout(share_only=1, inplace=1), pf.PF_EUNSUPPORTED)]:
        with pytest.raises(pf.PfError) as e:
            pf.pf_setup(*shape, lay)
        assert e.value.code == code


def test_null_handles():
    assert pf.pf_workspace_bytes(None) == 0
    pf.pf_destroy(None)
    assert pf.lib().pf_num_passes(None, 0) == pf.PF_EINVAL
    assert pf.lib().pf_copy(None, None, 16, None) == pf.PF_EINVAL
    assert pf.lib().pf_check_status(None) == pf.PF_EINVAL


def test_probe_arguments_are_checked_before_any_launch():
    """pf_probe refuses bad arguments on the host (the pointer values below are never dereferenced)."""
    L = pf.lib()
    assert L.pf_probe(pf.PF_PROBE_TILES, None, 256, 16, None) == pf.PF_EINVAL
    assert L.pf_probe(pf.PF_PROBE_TILES, 256, 264, 16, None) == pf.PF_EALIGN      # src not 16-byte aligned
    assert L.pf_probe(pf.PF_PROBE_TILES, 256, 512, 24, None) == pf.PF_EALIGN      # size not a multiple of 16
    assert L.pf_probe(pf.PF_PROBE_COPY, 256, 256, 16, None) == pf.PF_EALIAS       # copies need two buffers
    assert L.pf_probe(pf.PF_PROBE_TILES, 256, 256, 16, None) == pf.PF_EALIAS
    assert L.pf_probe(pf.PF_PROBE_TILES_INPLACE, 256, 512, 16, None) == pf.PF_EALIAS  # in place needs one
    assert L.pf_probe(7, 256, 512, 16, None) == pf.PF_EINVAL


def test_batch_setup_rejects_bad_arguments_before_touching_the_gpu():
    for dims, lay, tune, code in [
        ([], pf.Layout(), None, pf.PF_EINVAL),
        ([(16, 8, 8), (0, 8, 8)], pf.Layout(), None, pf.PF_EINVAL),
        ([(16, 8, 8), (22, 8, 8)], pf.Layout(), None, pf.PF_EUNSUPPORTED),  # factor 11
        ([(16, 8, 8)], pf.Layout(m1=2), None, pf.PF_EUNSUPPORTED),
        ([(16, 8, 8)], pf.Layout(inplace=1), None, pf.PF_EUNSUPPORTED),
        ([(16, 8, 8)], pf.Layout(math=pf.PF_MFMA_FP16X2), None, pf.PF_EUNSUPPORTED),
        ([(16, 8, 8)], pf.Layout(), [((0, 4, 0), (0, 0, 0))], pf.PF_EINVAL),  # radix order 4
        ([(16, 8, 8)], pf.Layout(), [((0, 0, 0), (0, -1, 0))], pf.PF_EINVAL),
    ]:
        with pytest.raises(pf.PfError) as e:
            pf.pf_batch_setup(dims, lay, tune)
        assert e.value.code == code, (dims, lay, tune)
    assert pf.pf_batch_bytes(None, 0) == 0
    assert pf.lib().pf_batch_set_mode(None, 1) == pf.PF_EINVAL
    assert pf.lib().pf_batch_ftran_r2c(None, None, None, None) == pf.PF_EINVAL


def test_cheb_third_transform_lengths():
    """Under the Chebyshev third transform z is transformed at length 2 (nz - 1): nz itself may be prime."""
    cheb = pf.Layout(third=pf.PF_THIRD_CHEB)
    assert pf.pf_check(16, 16, 17, cheb) == pf.PF_OK
    assert pf.pf_check(16, 16, 257, cheb) == pf.PF_OK
    assert pf.pf_check(16, 16, 17) == pf.PF_EUNSUPPORTED
    assert pf.pf_check(16, 16, 1, cheb) == pf.PF_EINVAL
    assert pf.pf_check(16, 16, 12, cheb) == pf.PF_EUNSUPPORTED  # 2 * 11


def test_empty_third_transform_takes_any_nz():
    """With the empty third transform nothing is transformed along z, so nz may
    have any prime factors (x and y still need 7-smooth lengths)."""
    empty = pf.Layout(third=pf.PF_THIRD_EMPTY)
    for nz in (17, 33, 1021):
        assert pf.pf_check(16, 16, nz, empty) == pf.PF_OK
        assert pf.pf_check(16, 16, nz) == pf.PF_EUNSUPPORTED
    assert pf.pf_check(16, 22, 17, empty) == pf.PF_EUNSUPPORTED  # y = 2 * 11
    assert pf.pf_check(16, 16, 8193, empty) == pf.PF_EUNSUPPORTED  # longer than a generic tile line
