"""CPU checks of the host construction of the red-black preconditioner
tables (built with g++ from the same header the library compiles): the
colour order against the oracle's 2-colouring, A's entries by colour
position, the Schur complement's column pattern against the sparsity of
F E computed here with SciPy (and each slot's transposed slot), and the tiles of black positions used by the
paired sweeps (a partition, each tile's halo exactly the columns its rows
reach outside it, every region-local column index in range and pointing at
the right position)."""
import ctypes
import os
import subprocess

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import precond as OP
from oracle.convdiff import convdiff_matrix
from paper_2312_02891_amd import workloads as WL

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def RB(tmp_path_factory):
    d = tmp_path_factory.mktemp("rb")
    so = str(d / "rb.so")
    srcs = [os.path.join(ROOT, "tests", "native", "selftest_rb.cpp"),
            os.path.join(ROOT, "paper_2312_02891_amd", "csrc", "gen.cpp")]
    subprocess.run(["g++", "-O2", "-shared", "-fPIC", "-std=c++17", "-pthread", "-ffp-contract=off",
                    "-o", so] + srcs, check=True)
    lib = ctypes.CDLL(so)
    lib.st_rb_ints.restype = ctypes.c_long
    lib.st_rb_doubles.restype = ctypes.c_long
    return lib


def build(RB, A, tiles):
    A = sp.csr_matrix(A)
    A.sort_indices()
    rp = np.ascontiguousarray(A.indptr, dtype=np.int32)
    ci = np.ascontiguousarray(A.indices, dtype=np.int32)
    v = np.ascontiguousarray(A.data, dtype=np.float64)
    info = np.zeros(7, dtype=np.int32)
    P = ctypes.c_void_p
    ok = RB.st_rb_build(ctypes.c_int(A.shape[0]), P(rp.ctypes.data), P(ci.ctypes.data), P(v.ctypes.data),
                        ctypes.c_int(tiles), P(info.ctypes.data))
    if not ok:
        return None
    out = dict(zip(["nred", "rbw", "t2w", "tile", "ntile", "maxreg", "nhalo"], info.tolist()))
    for name in ["rows", "pos", "eci", "t2ci", "t2rev", "t2lc", "halo_off", "halo", "halo_ci"]:
        k = RB.st_rb_ints(name.encode(), None)
        a = np.zeros(k, dtype=np.int32)
        RB.st_rb_ints(name.encode(), P(a.ctypes.data))
        out[name] = a
    for name in ["dg", "eval", "etv"]:
        k = RB.st_rb_doubles(name.encode(), None)
        a = np.zeros(k, dtype=np.float64)
        RB.st_rb_doubles(name.encode(), P(a.ctypes.data))
        out[name] = a
    return out


def rows_per_wg(n):
    r = (n + 511) // 512
    r = ((r + 255) // 256) * 256
    return max(256, min(r, 8192))


CASES = [(2, 9, (7.0, -3.0), 4), (2, 24, (50.0, 20.0), 5), (3, 7, (2.0, 5.0, -1.0), 3),
         (2, 64, (10.0, -4.0), None), (3, 16, (1.0, 2.0, 3.0), None), (2, 1, (1.0, 1.0), 1)]


@pytest.mark.parametrize("dim,N,omega,tiles", CASES)
def test_tables_against_definitions(RB, dim, N, omega, tiles):
    A = sp.csr_matrix(convdiff_matrix(dim, N, omega))
    n = A.shape[0]
    if tiles is None:
        tiles = (n + rows_per_wg(n) - 1) // rows_per_wg(n)
    h = build(RB, A, tiles)
    col = OP.two_coloring(A)
    red = np.where(col == 0)[0]
    blk_nat = np.where(col == 1)[0]
    nr, nb = len(red), len(blk_nat)
    assert h["nred"] == nr
    rows, pos = h["rows"], h["pos"]
    # red rows ascending, black rows a permutation of the black set
    assert np.array_equal(rows[:nr], red)
    assert np.array_equal(np.sort(rows[nr:]), blk_nat)
    assert np.array_equal(pos[rows], np.arange(n))
    blk = rows[nr:]
    # diagonal and slot tables by colour position
    assert np.array_equal(h["dg"], A.diagonal())
    W = h["rbw"]
    eci = h["eci"].reshape(W, n)
    ev = h["eval"].reshape(W, n)
    et = h["etv"].reshape(W, n)
    Ad = A.toarray() if n <= 4096 else None
    for p in range(0, n, max(1, n // 300)):
        i = rows[p]
        used = eci[:, p] != i
        want = sorted(c for c in A.indices[A.indptr[i]:A.indptr[i + 1]] if c != i)
        assert sorted(eci[used, p].tolist()) == want
        for u in np.where(used)[0]:
            c = eci[u, p]
            assert ev[u, p] == A[i, c] and et[u, p] == A[c, i]
        assert np.all(ev[~used, p] == 0) and np.all(et[~used, p] == 0)
    if nb == 0:
        return
    # Schur pattern: off-diagonal nonzero pattern of F E (F: black x red,
    # E: red x black), in the tile order of the black positions
    S = abs(A)
    F = S[blk][:, red]
    E = S[red][:, blk]
    Tp = (F @ E).tocsr()
    Tp.setdiag(0)
    Tp.eliminate_zeros()
    W2 = h["t2w"]
    t2ci = h["t2ci"].reshape(W2, nb)
    for pb in range(nb):
        cols = t2ci[:, pb]
        used = cols[cols != pb]
        assert len(set(used.tolist())) == len(used)
        assert sorted(used.tolist()) == sorted(Tp.indices[Tp.indptr[pb]:Tp.indptr[pb + 1]].tolist())
    assert W2 == max(1, max(np.diff(Tp.indptr)))
    # the transposed entry's slot: column pb in row c's slots (the pattern of
    # T is symmetric here), -1 on unused slots
    t2rev = h["t2rev"].reshape(W2, nb)
    for pb in range(nb):
        for q in range(W2):
            c = t2ci[q, pb]
            if c == pb:
                assert t2rev[q, pb] == -1
            else:
                assert t2rev[q, pb] >= 0 and t2ci[t2rev[q, pb], c] == pb
    # tiles: consecutive ranges of `tile`, rows ascending inside each
    tile, ntile = h["tile"], h["ntile"]
    assert tile == (nb + tiles - 1) // tiles and ntile == (nb + tile - 1) // tile
    t2lc = h["t2lc"].reshape(W2, nb)
    off, halo = h["halo_off"], h["halo"]
    assert len(off) == ntile + 1 and off[0] == 0 and off[-1] == len(halo) == h["nhalo"]
    maxreg = 0
    for t in range(ntile):
        p0, p1 = t * tile, min(nb, (t + 1) * tile)
        nin = p1 - p0
        assert np.all(np.diff(blk[p0:p1]) > 0)
        hl = halo[off[t]:off[t + 1]]
        region = np.concatenate([np.arange(p0, p1), hl])
        cols = t2ci[:, p0:p1]
        outside = sorted(set(cols[(cols < p0) | (cols >= p1)].tolist()))
        assert hl.tolist() == outside
        lc = t2lc[:, p0:p1]
        assert lc.min() >= 0 and lc.max() < nin + len(hl)
        assert np.array_equal(region[lc], cols)
        maxreg = max(maxreg, nin + len(hl))
    assert h["maxreg"] == maxreg
    # the halo rows' columns, copied per halo entry
    nh = len(halo)
    hci = h["halo_ci"].reshape(W2, max(nh, 1))[:, :nh]
    assert np.array_equal(hci, t2ci[:, halo])


def test_without_tiles_black_rows_stay_ascending(RB):
    """tiles = 0 (matrices below the pairing size): the black rows keep
    their ascending order, no tiles or halos are made, and T's columns are
    the same pattern as with tiles."""
    A = convdiff_matrix(2, 24, (50.0, 20.0))
    h = build(RB, A, 0)
    col = OP.two_coloring(A)
    nr = h["nred"]
    assert np.array_equal(h["rows"][nr:], np.where(col == 1)[0])
    assert h["tile"] == 0 and h["ntile"] == 0 and h["nhalo"] == 0 and h["halo_off"].tolist() == [0]
    t = build(RB, A, 5)
    nb = A.shape[0] - nr
    W2 = h["t2w"]
    pat = lambda hh: sorted(tuple(sorted(hh["rows"][nr + hh["t2ci"].reshape(W2, nb)[:, p]].tolist()))
                            for p in range(nb))
    assert t["t2w"] == W2 and pat(h) == pat(t)


def test_tiles_of_a_grid_are_compact(RB):
    """On the 2-D 256^2 grid with one tile per row workgroup (128 black
    rows) the regions hold at most 1.6 times the black rows: the breadth
    first tiles are compact (strips of the natural order would need 5)."""
    A = convdiff_matrix(2, 256, (50.0, 20.0))
    n = A.shape[0]
    h = build(RB, A, (n + rows_per_wg(n) - 1) // rows_per_wg(n))
    nb = n - h["nred"]
    assert h["tile"] == 128
    assert (nb + h["nhalo"]) / nb < 1.6
    assert h["maxreg"] * 4 * 8 <= 64 * 1024


def test_non_bipartite_is_rejected(RB):
    rp, ci, v = WL.mass_csr(2, 5)
    M = sp.csr_matrix((v, ci, rp), shape=(25, 25))
    assert build(RB, M, 1) is None
